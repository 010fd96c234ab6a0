"""Host-side checks of the sweep-block tuning table: the autotune module's range merging and
header text, and the committed table the library is built with."""
import os
import re

from paper_1605_08771_amd import autotune as at

ROW = re.compile(r"\{(\d+), (\d+), (\d+)\}")


def _rows(text):
    body = text[text.index("kSweepTune[]"):]
    return [tuple(int(v) for v in m) for m in ROW.findall(body)]


def test_rows_from_midpoints_and_merging():
    choice = [(256, 64), (384, 64), (512, 128), (768, 256), (1024, 256), (2048, 512)]
    assert at.rows_from(choice) == [(447, 64), (639, 128), (1535, 256), (2048, 512)]
    assert at.rows_from([(300, 128)]) == [(300, 128)]


def test_header_round_trip():
    table = [(0, [(447, 64), (2048, 256)]), (1, [(1000, 128)])]
    text = at.header(table, "test device", 3)
    assert _rows(text) == [(0, 447, 64), (0, 2048, 256), (1, 1000, 128)]
    assert "#pragma once" in text and "namespace feast" in text


def test_committed_table_is_well_formed():
    path = os.path.join(os.path.dirname(at.__file__), "csrc", "sweep_tune.h")
    rows = _rows(open(path).read())
    assert rows
    for cls in (0, 1):
        mine = [r for r in rows if r[0] == cls]
        assert mine, cls
        n_max = [r[1] for r in mine]
        assert n_max == sorted(n_max) and len(set(n_max)) == len(n_max)
        assert all(r[2] in (64, 128, 256, 512) for r in mine)
