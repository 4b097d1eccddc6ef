// cell_table.h -- cell edges (units, x y z) per grain-density bucket, used
// when a context leaves its cell edges to the library. Bucket b holds views
// with at least 0.75 * 2^(b-1) grains per 1000 um^3 (b = 0: fewer than
// 0.75). Written by paper_1311_5334_amd/autotune.py from timings of the
// whole path on synthetic views at each bucket's middle density:
//   bucket 1: 1.06 grains/1000um^3, 31587 grains in 8 views; best (250, 1500, 500) 0.929 ms, default (250, 750, 500) 0.980 ms, worst 1.206 ms
//   bucket 2: 2.12 grains/1000um^3, 51449 grains in 8 views; best (150, 500, 200) 1.163 ms, default (250, 750, 500) 1.361 ms, worst 1.662 ms
//   bucket 3: 4.24 grains/1000um^3, 102475 grains in 8 views; best (100, 500, 300) 3.203 ms, default (250, 750, 500) 3.296 ms, worst 4.246 ms
//   bucket 4: 8.49 grains/1000um^3, 205515 grains in 8 views; best (100, 1000, 500) 10.560 ms, default (250, 750, 500) 10.866 ms, worst 16.490 ms
//   bucket 5: 16.97 grains/1000um^3, 411290 grains in 8 views; best (150, 400, 200) 102.377 ms, default (250, 750, 500) 111.385 ms, worst 166.225 ms
#ifndef EMT_CELL_TABLE_H
#define EMT_CELL_TABLE_H

namespace emt {

constexpr int kTunedCells[8][3] = {
    {250, 1500, 500},  // bucket 0
    {250, 1500, 500},  // bucket 1
    {150, 500, 200},  // bucket 2
    {100, 500, 300},  // bucket 3
    {100, 1000, 500},  // bucket 4
    {150, 400, 200},  // bucket 5
    {150, 400, 200},  // bucket 6
    {150, 400, 200},  // bucket 7
};

}  // namespace emt

#endif
