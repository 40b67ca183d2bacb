"""The multisection tuning table on the device: a new handle holds the table
the library was built with, the table can be replaced, cleared and restored,
a solve takes its multisection shape from it (mr3_stats reports the key and
the lanes), and results under different shapes pass the same oracle gates."""
import os

import pytest
import torch

import workloads as W
from paper_1304_1864_amd import tune
from tests.test_gpu_parity import run_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr3():
    import paper_1304_1864_amd as lib

    lib.load_library()
    return lib


def test_handle_starts_with_builtin_table(mr3):
    inc = os.path.join(os.path.dirname(mr3.__file__), "csrc", "tuning_gfx950.inc")
    h = mr3.Handle(0)
    assert h.tuning() == tune.parse(open(inc).read())
    h.close()


def test_set_get_restore_and_lookup(mr3):
    h = mr3.Handle(0)
    R, C = mr3.MR3_TUNE_ROOT, mr3.MR3_TUNE_CHILD
    table = [(R, 64, 1024, 2048, 512, 1024, 6), (C, 32, 16, 32, 256, 512, 24)]
    h.set_tuning(table)
    assert h.tuning() == table
    assert h.bisect_lanes(R, 64, 1500, 600) == 6
    assert h.bisect_lanes(R, 64, 2048, 600) == 0   # count_hi is exclusive
    assert h.bisect_lanes(R, 32, 1500, 600) == 0   # other precision
    assert h.bisect_lanes(C, 32, 20, 300) == 24
    h.set_params(precision=64, lanes_per_eig=5)     # the override wins (largest candidate <= 5)
    assert h.bisect_lanes(R, 64, 1500, 600) == 4
    h.reset_params()
    for bad in ([(2, 64, 1, 2, 1, 2, 4)], [(R, 16, 1, 2, 1, 2, 4)], [(R, 64, 2, 2, 1, 2, 4)],
                [(R, 64, 1, 2, 1, 2, 5)]):
        with pytest.raises(mr3.MR3Error):
            h.set_tuning(bad)
    assert h.tuning() == table                      # unchanged after a refused table
    h.set_tuning([])
    assert h.tuning() == [] and h.bisect_lanes(R, 64, 1500, 600) == 0
    h.set_tuning(None)
    assert h.tuning() == mr3.Handle(0).tuning()
    with pytest.raises(mr3.MR3Error):
        h.bisect_lanes(3, 64, 1, 1)
    h.close()


def test_solve_takes_the_table_shape(mr3):
    """A table entry for this problem's keys decides the staged shapes of
    both stages; two different tables give results within the same gates."""
    d, e, _ = W.prescribed_spectrum(3000, 7)
    h = mr3.Handle(0)
    h.set_tuning([])
    run_case(mr3, d, e, handle=h, check_angles=False)
    st = h.stats()
    kr = (st["bisect_count"][0], st["bisect_rows"][0])
    kc = (st["bisect_count"][1], st["bisect_rows"][1])
    assert kr == (3000, 3000)
    assert kc[0] > 0, "the case must have clusters"
    for lr, lc in ((2, 32), (12, 4)):
        h.set_tuning([(0, 64) + tune.bucket(kr[0]) + tune.bucket(kr[1]) + (lr,),
                      (1, 64) + tune.bucket(kc[0]) + tune.bucket(kc[1]) + (lc,)])
        run_case(mr3, d, e, handle=h, check_angles=(lr == 2))
        st = h.stats()
        assert st["bisect_lanes"][0] == lr
        assert st["bisect_lanes"][1] == lc
    torch.cuda.synchronize()
    h.close()
