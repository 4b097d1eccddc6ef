// cell_table.h -- cell edges (units, x y z) per grain-density bucket, used
// when a context leaves its cell edges to the library. Bucket b holds views
// with at least 0.75 * 2^(b-1) grains per 1000 um^3 (b = 0: fewer than
// 0.75). Written by paper_1311_5334_amd/autotune.py from timings of the
// whole path on synthetic views at each bucket's middle density:
//   bucket 1: 1.06 grains/1000um^3, 31587 grains in 8 views; best (200, 400, 300) 1.090 ms, default (250, 750, 500) 1.197 ms, worst 1.484 ms
//   bucket 2: 2.12 grains/1000um^3, 51449 grains in 8 views; best (150, 400, 300) 1.382 ms, default (250, 750, 500) 1.736 ms, worst 2.263 ms
//   bucket 3: 4.24 grains/1000um^3, 102475 grains in 8 views; best (200, 750, 500) 3.271 ms, default (250, 750, 500) 3.317 ms, worst 6.015 ms
//   bucket 4: 8.49 grains/1000um^3, 205515 grains in 8 views; best (150, 750, 300) 13.089 ms, default (250, 750, 500) 14.455 ms, worst 28.076 ms
//   bucket 5: 16.97 grains/1000um^3, 411290 grains in 8 views; best (200, 750, 300) 131.239 ms, default (250, 750, 500) 156.603 ms, worst 255.575 ms
#ifndef EMT_CELL_TABLE_H
#define EMT_CELL_TABLE_H

namespace emt {

constexpr int kTunedCells[8][3] = {
    {200, 400, 300},  // bucket 0
    {200, 400, 300},  // bucket 1
    {150, 400, 300},  // bucket 2
    {200, 750, 500},  // bucket 3
    {150, 750, 300},  // bucket 4
    {200, 750, 300},  // bucket 5
    {200, 750, 300},  // bucket 6
    {200, 750, 300},  // bucket 7
};

}  // namespace emt

#endif
