"""The multisection tuning table on the host: the table compiled into the
library parses, every entry is one the library accepts (known stage and
precision, non-empty power-of-two ranges, a lane count the staged kernel
has), keys do not overlap, and the tuner's writer and reader agree."""
import os

import paper_1304_1864_amd as mr3
from paper_1304_1864_amd import tune

INC = os.path.join(os.path.dirname(mr3.__file__), "csrc", "tuning_gfx950.inc")


def test_builtin_table_entries_are_valid():
    entries = tune.parse(open(INC).read())
    seen = set()
    for st, prec, c0, c1, r0, r1, lanes in entries:
        assert st in (mr3.MR3_TUNE_ROOT, mr3.MR3_TUNE_CHILD)
        assert prec in (32, 64)
        assert 1 <= c0 < c1 and 1 <= r0 < r1
        assert (c0, c1) == tune.bucket(c0) and (r0, r1) == tune.bucket(r0)
        assert lanes in mr3.LANE_CANDIDATES
        assert (st, prec, c0, r0) not in seen
        seen.add((st, prec, c0, r0))


def test_bucket():
    assert tune.bucket(1) == (1, 2)
    assert tune.bucket(20000) == (16384, 32768)
    assert tune.bucket(16384) == (16384, 32768)
    assert tune.bucket(16383) == (8192, 16384)


def test_render_parse_round_trip():
    entries = [(0, 64, 16384, 32768, 16384, 32768, 6), (1, 32, 1024, 2048, 256, 512, 24)]
    text = tune.render(entries, ["device: test"])
    assert tune.parse(text) == entries
    assert all(line.startswith("//") or line.startswith("MR3_TUNE(") for line in text.splitlines())


def test_choose_prefers_fewer_lanes_within_noise():
    assert tune.choose({1: 10.0, 2: 5.0, 4: 4.95, 8: 6.0}) == 2
    assert tune.choose({1: 10.0, 2: 5.0, 4: 4.0}) == 4
