"""Host logic of the autotuner (no GPU): the tables it writes must keep every
constant the kernels read, the in-tree tables must parse, and the tile
search must start from the values in force."""
import os
import re

from paper_1311_5334_amd import autotune as at

CSRC = os.path.join(os.path.dirname(at.TILE_TABLE))


def _defines(text: str) -> dict:
    return {m.group(1): m.group(2) for m in re.finditer(r"#define (EMT_\w+) (.+?)(?:\s+//.*)?$",
                                                         text, re.M)}


def test_tile_table_round_trip(tmp_path):
    tiles = at.read_tiles()
    assert set(tiles) == set(at.TILE_SPACE)
    out = tmp_path / "tile_table.h"
    at.write_tiles(str(out), tiles, "//   test")
    assert at.read_tiles(str(out)) == tiles
    # the written header defines everything the in-tree one does (the
    # derived queue capacities included), with the same values
    assert _defines(out.read_text()) == _defines(open(at.TILE_TABLE).read())


def test_every_tile_constant_the_kernels_use_is_tuned():
    used = set()
    for f in os.listdir(CSRC):
        if f.endswith((".hip", ".h")) and f != "tile_table.h":
            used |= set(re.findall(r"\b(EMT_(?:COUNT|CHUNK|FLUSH|MERGE_WIDE|CELLS_PER)\w*)\b",
                                   open(os.path.join(CSRC, f)).read()))
    derived = {"EMT_COUNT_PIECE_CAP", "EMT_COUNT_RUN_CAP"}
    assert used - derived <= set(at.TILE_SPACE), used - derived - set(at.TILE_SPACE)


def test_tile_candidates_are_the_start_and_one_at_a_time_variations():
    start = at.read_tiles()
    cands = at.tile_candidates(start)
    assert cands[0] == start
    assert len(cands) == 1 + sum(len([v for v in vals if v != start[k]])
                                 for k, vals in at.TILE_SPACE.items())
    for c in cands[1:]:
        changed = [k for k in c if c[k] != start[k]]
        assert len(changed) == 1 and c[changed[0]] in at.TILE_SPACE[changed[0]]
    assert len({at._tag(c) for c in cands}) == len(cands)


def test_cell_table_parses_and_write_table_round_trips(tmp_path):
    text = open(at.TABLE).read()
    rows = [tuple(int(x) for x in m.groups())
            for m in re.finditer(r"\{(\d+), (\d+), (\d+)\},\s+// bucket \d", text)]
    assert len(rows) == at.N_BUCKETS
    assert all(0 < e <= 1 << 18 for r in rows for e in r)
    best = {b: rows[b] for b in at.TUNED}
    out = tmp_path / "cell_table.h"
    at.write_table(str(out), best, "//   test")
    again = [tuple(int(x) for x in m.groups())
             for m in re.finditer(r"\{(\d+), (\d+), (\d+)\},\s+// bucket \d", out.read_text())]
    # buckets outside the tuned range copy the nearest tuned one
    assert again == [rows[min(max(b, min(at.TUNED)), max(at.TUNED))] for b in range(at.N_BUCKETS)]
