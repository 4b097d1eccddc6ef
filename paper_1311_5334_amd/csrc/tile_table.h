// tile_table.h -- queue sizes and launch shapes of the counting kernel and
// the cell budget per grain, chosen by paper_1311_5334_amd/autotune.py
// --tiles from timings of the whole path; -D on the compiler line overrides
// each value.
//   starting tiles {'EMT_COUNT_PIECE': 3, 'EMT_COUNT_LANE_PIECES': 24, 'EMT_COUNT_FETCH': 6, 'EMT_COUNT_REFILL': 32, 'EMT_FLUSH_UNROLL': 1, 'EMT_CHUNK_SEEDS': 128, 'EMT_COUNT_BLOCKS': 1024, 'EMT_COUNT_OCCUPANCY': 5, 'EMT_MERGE_WIDE': 16, 'EMT_CELLS_PER_GRAIN': 4}: c2 1.054 ms, c5x8 36.628 ms, c3x16 5.363 ms
//   chosen tiles {'EMT_COUNT_PIECE': 3, 'EMT_COUNT_LANE_PIECES': 24, 'EMT_COUNT_FETCH': 6, 'EMT_COUNT_REFILL': 32, 'EMT_FLUSH_UNROLL': 1, 'EMT_CHUNK_SEEDS': 128, 'EMT_COUNT_BLOCKS': 1024, 'EMT_COUNT_OCCUPANCY': 5, 'EMT_MERGE_WIDE': 16, 'EMT_CELLS_PER_GRAIN': 4} (each constant's best one-at-a-time variation)
//   16 builds timed
#ifndef EMT_TILE_TABLE_H
#define EMT_TILE_TABLE_H

#ifndef EMT_COUNT_PIECE
#define EMT_COUNT_PIECE 3  // grains a flush lane tests per queue entry
#endif
#ifndef EMT_COUNT_LANE_PIECES
#define EMT_COUNT_LANE_PIECES 24  // queue entries a lane adds per step
#endif
#ifndef EMT_COUNT_FETCH
#define EMT_COUNT_FETCH 6  // cell pencils a lane fetches per step
#endif
#ifndef EMT_COUNT_REFILL
#define EMT_COUNT_REFILL 32  // lanes waiting for a seed before a wave refills
#endif
#ifndef EMT_FLUSH_UNROLL
#define EMT_FLUSH_UNROLL 1  // queue words a flush trip loads before testing
#endif
#ifndef EMT_CHUNK_SEEDS
#define EMT_CHUNK_SEEDS 128  // seeds a wave takes at a time (single views)
#endif
#ifndef EMT_COUNT_BLOCKS
#define EMT_COUNT_BLOCKS 1024  // workgroups of the counting kernel
#endif
#ifndef EMT_COUNT_OCCUPANCY
#define EMT_COUNT_OCCUPANCY 5  // waves per SIMD the counting kernel is compiled for
#endif
#ifndef EMT_MERGE_WIDE
#define EMT_MERGE_WIDE 16  // grid-wide merge rounds at most before the per-view tails
#endif
#ifndef EMT_CELLS_PER_GRAIN
#define EMT_CELLS_PER_GRAIN 4  // cells a view may use per grain (plus 4096)
#endif

// queue capacities that follow from the above
#ifndef EMT_COUNT_PIECE_CAP
#define EMT_COUNT_PIECE_CAP (128 * EMT_COUNT_LANE_PIECES)
#endif
#ifndef EMT_COUNT_RUN_CAP
#define EMT_COUNT_RUN_CAP (64 * EMT_COUNT_FETCH)
#endif

#endif
