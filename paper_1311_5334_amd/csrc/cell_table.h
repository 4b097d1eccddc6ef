// cell_table.h -- cell edges (units, x y z) per grain-density bucket, used
// when a context leaves its cell edges to the library. Bucket b holds views
// with at least 0.75 * 2^(b-1) grains per 1000 um^3 (b = 0: fewer than
// 0.75). Written by paper_1311_5334_amd/autotune.py from timings of the
// whole path on synthetic views at each bucket's middle density:
//   bucket 1: 1.06 grains/1000um^3, 31587 grains in 8 views; best (200, 2000, 800) 0.824 ms, default (250, 750, 500) 0.847 ms, worst 0.994 ms
//   bucket 2: 2.12 grains/1000um^3, 51449 grains in 8 views; best (150, 1500, 800) 0.999 ms, default (250, 750, 500) 1.076 ms, worst 1.229 ms
//   bucket 3: 4.24 grains/1000um^3, 102475 grains in 8 views; best (150, 1500, 800) 2.430 ms, default (250, 750, 500) 2.606 ms, worst 3.383 ms
//   bucket 4: 8.49 grains/1000um^3, 205515 grains in 8 views; best (100, 1000, 500) 8.209 ms, default (250, 750, 500) 8.680 ms, worst 15.901 ms
//   bucket 5: 16.97 grains/1000um^3, 411290 grains in 8 views; best (100, 750, 800) 77.197 ms, default (250, 750, 500) 89.158 ms, worst 156.366 ms
#ifndef EMT_CELL_TABLE_H
#define EMT_CELL_TABLE_H

namespace emt {

constexpr int kTunedCells[8][3] = {
    {200, 2000, 800},  // bucket 0
    {200, 2000, 800},  // bucket 1
    {150, 1500, 800},  // bucket 2
    {150, 1500, 800},  // bucket 3
    {100, 1000, 500},  // bucket 4
    {100, 750, 800},  // bucket 5
    {100, 750, 800},  // bucket 6
    {100, 750, 800},  // bucket 7
};

}  // namespace emt

#endif
