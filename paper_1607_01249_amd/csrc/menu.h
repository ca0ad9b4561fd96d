// Tile shapes the library instantiates, per dtype and kernel family.
//
// Sec. 2.2 blocks each tile edge by b in {w, 2w, 3w, 4w}.  Here w = 16
// elements for both data types (64 B of FP32, one 128-B line of FP64), so the
// regular moved-family tiles are {16,32,48,64} x {16,32,48,64}.  For indices
// shorter than w the remainder rule of Sec. 2.3 would waste most of a tile,
// so skinny shapes pair a short edge with a long one; long-run shapes (512-B
// FP32 and 1-KiB FP64 runs along one side) trade the other edge for fewer
// DRAM pages per tile.  Preserved-family
// tiles copy rows that are contiguous in both tensors; they are sized by
// the number of elements a workgroup moves (1K to 4K).
#pragma once

// Single complex elements (8 bytes) use the FP64 menus.  Double complex
// elements are 16 bytes, one vector each: w = 8 elements (one 128-B line),
// regular tiles {8,16,24,32} x {8,16,24,32}, skinny shapes for 2- and
// 4-element edges and 1-KiB long-run shapes.
//
// X(tile_a, tile_b)
#define TTX_MOVED_MENU_F32(X)                                                             \
    X(16, 16) X(16, 32) X(16, 48) X(16, 64) X(32, 16) X(32, 32) X(32, 48) X(32, 64)       \
    X(48, 16) X(48, 32) X(48, 48) X(48, 64) X(64, 16) X(64, 32) X(64, 48) X(64, 64)       \
    X(4, 256) X(8, 128) X(256, 4) X(128, 8) X(128, 32) X(32, 128)

#define TTX_MOVED_MENU_F64(X)                                                             \
    X(16, 16) X(16, 32) X(16, 48) X(16, 64) X(32, 16) X(32, 32) X(32, 48) X(32, 64)       \
    X(48, 16) X(48, 32) X(48, 48) X(48, 64) X(64, 16) X(64, 32) X(64, 48) X(64, 64)       \
    X(2, 256) X(4, 128) X(256, 2) X(128, 4) X(128, 16) X(16, 128)

#define TTX_MOVED_MENU_C64(X)                                                             \
    X(8, 8) X(8, 16) X(8, 24) X(8, 32) X(16, 8) X(16, 16) X(16, 24) X(16, 32)              \
    X(24, 8) X(24, 16) X(24, 24) X(24, 32) X(32, 8) X(32, 16) X(32, 24) X(32, 32)          \
    X(2, 128) X(4, 64) X(128, 2) X(64, 4) X(64, 16) X(16, 64)

// Larger moved-family tiles, compiled only at run time as size-specialised
// kernels (no pre-compiled instance): runs of 256 to 512 bytes on both sides,
// for the shape search around the tuner's fastest blockings.  X(tile_a, tile_b)
#define TTX_MOVED_LARGE_F32(X) X(64, 128) X(128, 64) X(96, 128) X(128, 96)
#define TTX_MOVED_LARGE_F64(X) X(32, 128) X(128, 32) X(64, 96) X(96, 64)
#define TTX_MOVED_LARGE_C64(X) X(32, 64) X(64, 32) X(48, 64) X(64, 48)

// X(tile_a, rows)
#define TTX_PRESERVED_MENU_F32(X)                                                         \
    X(16, 64) X(16, 256) X(32, 32) X(32, 128) X(64, 16) X(64, 64) X(128, 8) X(128, 32)    \
    X(256, 4) X(256, 16) X(4, 256) X(8, 256)

#define TTX_PRESERVED_MENU_F64(X)                                                         \
    X(16, 64) X(16, 256) X(32, 32) X(32, 128) X(64, 16) X(64, 64) X(128, 8) X(128, 32)    \
    X(256, 4) X(256, 16) X(2, 512) X(4, 256)

#define TTX_PRESERVED_MENU_C64(X)                                                         \
    X(8, 64) X(8, 256) X(16, 32) X(16, 128) X(32, 16) X(32, 64) X(64, 8) X(64, 32)        \
    X(128, 4) X(128, 16) X(2, 256) X(4, 128)

// Staged preserved-family tiles, for short stride-1 rows: X(n0_max, tile_x,
// tile_y) with n0_max lanes per row (rows of n0 <= n0_max elements), tile_x
// rows along A's next indices and tile_y along B's next indices.
#define TTX_STAGED_MENU_F32(X)                                                            \
    X(16, 16, 16) X(16, 8, 32) X(16, 32, 8) X(32, 8, 16) X(32, 16, 8) X(32, 4, 32)        \
    X(32, 32, 4) X(32, 8, 8) X(64, 8, 8) X(64, 4, 16) X(64, 16, 4) X(64, 4, 4)

#define TTX_STAGED_MENU_F64(X)                                                            \
    X(16, 16, 8) X(16, 8, 16) X(16, 4, 32) X(16, 32, 4) X(32, 8, 8) X(32, 4, 16)          \
    X(32, 16, 4) X(32, 2, 32) X(32, 32, 2) X(64, 4, 8) X(64, 8, 4) X(64, 4, 4)

// Double complex rows are staged only when shorter than 16 elements (256 B).
#define TTX_STAGED_MENU_C64(X)                                                            \
    X(16, 8, 8) X(16, 4, 16) X(16, 16, 4) X(16, 2, 32) X(16, 32, 2) X(16, 4, 8)           \
    X(16, 8, 4) X(16, 4, 4) X(16, 2, 16) X(16, 16, 2)

// Dense tiles: elements per tile (4 KiB FP32, 8 KiB FP64 and single complex,
// 8 KiB double complex).
#define TTX_DENSE_CAP_F32 1024
#define TTX_DENSE_CAP_F64 1024
#define TTX_DENSE_CAP_C32 1024
#define TTX_DENSE_CAP_C64 512
// and for whole units of kept rows: 16-byte units (8 KiB), 8-byte units (8 KiB)
#define TTX_DENSE_CAP_W16 512
#define TTX_DENSE_CAP_W8 1024

// Tile variants compiled into the persistent batched kernel, per dtype:
// X(index, kind, p1, p2, p3).  For the moved, preserved and flat kinds
// (TTX_FAMILY_*) p1 x p2 is the tile and p3 = 1 selects 16-byte accesses on
// both sides (flat tiles: p1 consecutive elements, four per thread, in
// vectors or single elements); for TTX_BATCH_STAGED p1 is the row-lane count and p2 x p3 the
// staged tile; for TTX_BATCH_DENSE p1 is the dense capacity.  Kept small: every variant adds code to the one kernel and
// its register and LDS needs set the kernel's occupancy (the dense variant sets the
// registers; the large vector tiles, 16-17 KB of LDS like it, cost no occupancy and carry
// most of the batch's bytes: its largest problems run 2-3% faster with them).
#define TTX_BATCH_STAGED 4
#define TTX_BATCH_DENSE 5

#define TTX_BATCH_MENU_F32(X)                                                             \
    X(0, TTX_FAMILY_MOVED, 64, 32, 1) X(1, TTX_FAMILY_MOVED, 32, 32, 1)                   \
    X(2, TTX_FAMILY_MOVED, 32, 64, 1) X(3, TTX_FAMILY_MOVED, 32, 32, 0)                   \
    X(4, TTX_FAMILY_MOVED, 8, 128, 0) X(5, TTX_FAMILY_MOVED, 128, 8, 0)                   \
    X(6, TTX_FAMILY_PRESERVED, 64, 16, 1) X(7, TTX_FAMILY_PRESERVED, 64, 16, 0)           \
    X(8, TTX_FAMILY_PRESERVED, 16, 64, 0) X(9, TTX_FAMILY_FLAT, 4096, 1, 1)               \
    X(10, TTX_FAMILY_FLAT, 1024, 1, 0) X(11, TTX_BATCH_STAGED, 16, 8, 8)                  \
    X(12, TTX_BATCH_STAGED, 32, 8, 8) X(13, TTX_BATCH_STAGED, 64, 4, 4)                   \
    X(14, TTX_BATCH_DENSE, TTX_DENSE_CAP_F32, 0, 0) X(15, TTX_FAMILY_MOVED, 64, 64, 1)     \
    X(16, TTX_FAMILY_MOVED, 128, 32, 1) X(17, TTX_FAMILY_MOVED, 32, 128, 1)

#define TTX_BATCH_MENU_F64(X)                                                             \
    X(0, TTX_FAMILY_MOVED, 32, 32, 1) X(1, TTX_FAMILY_MOVED, 32, 16, 1)                   \
    X(2, TTX_FAMILY_MOVED, 16, 32, 1) X(3, TTX_FAMILY_MOVED, 32, 32, 0)                   \
    X(4, TTX_FAMILY_MOVED, 4, 128, 0) X(5, TTX_FAMILY_MOVED, 128, 4, 0)                   \
    X(6, TTX_FAMILY_PRESERVED, 64, 16, 1) X(7, TTX_FAMILY_PRESERVED, 64, 16, 0)           \
    X(8, TTX_FAMILY_PRESERVED, 16, 64, 0) X(9, TTX_FAMILY_FLAT, 2048, 1, 1)               \
    X(10, TTX_FAMILY_FLAT, 1024, 1, 0) X(11, TTX_BATCH_STAGED, 16, 8, 8)                  \
    X(12, TTX_BATCH_STAGED, 32, 4, 4) X(13, TTX_BATCH_STAGED, 64, 4, 4)                   \
    X(14, TTX_BATCH_DENSE, TTX_DENSE_CAP_F64, 0, 0) X(15, TTX_FAMILY_MOVED, 64, 32, 1)     \
    X(16, TTX_FAMILY_MOVED, 32, 64, 1) X(17, TTX_FAMILY_MOVED, 16, 128, 1)

#define TTX_BATCH_MENU_SIZE 18
