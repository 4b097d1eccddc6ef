// cell_table.h -- cell edges (units, x y z) per grain-density bucket, used
// when a context leaves its cell edges to the library. Bucket b holds views
// with at least 0.75 * 2^(b-1) grains per 1000 um^3 (b = 0: fewer than
// 0.75). Written by paper_1311_5334_amd/autotune.py from timings of the
// whole path on synthetic views at each bucket's middle density:
//   bucket 1: 1.06 grains/1000um^3, 31587 grains in 8 views; best (150, 750, 300) 0.894 ms, default (250, 750, 500) 0.931 ms, worst 1.064 ms
//   bucket 2: 2.12 grains/1000um^3, 51449 grains in 8 views; best (100, 750, 300) 1.148 ms, default (250, 750, 500) 1.233 ms, worst 1.406 ms
//   bucket 3: 4.24 grains/1000um^3, 102475 grains in 8 views; best (100, 1000, 800) 2.912 ms, default (250, 750, 500) 3.018 ms, worst 3.879 ms
//   bucket 4: 8.49 grains/1000um^3, 205515 grains in 8 views; best (150, 1000, 500) 10.084 ms, default (250, 750, 500) 10.616 ms, worst 15.565 ms
//   bucket 5: 16.97 grains/1000um^3, 411290 grains in 8 views; best (100, 750, 200) 87.134 ms, default (250, 750, 500) 88.904 ms, worst 119.788 ms
#ifndef EMT_CELL_TABLE_H
#define EMT_CELL_TABLE_H

namespace emt {

constexpr int kTunedCells[8][3] = {
    {150, 750, 300},  // bucket 0
    {150, 750, 300},  // bucket 1
    {100, 750, 300},  // bucket 2
    {100, 1000, 800},  // bucket 3
    {150, 1000, 500},  // bucket 4
    {100, 750, 200},  // bucket 5
    {100, 750, 200},  // bucket 6
    {100, 750, 200},  // bucket 7
};

}  // namespace emt

#endif
