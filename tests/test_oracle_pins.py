"""The CPU oracle against facts that do not come from it (CPU only)."""
import os

import pytest

import oracle
from tests import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    ok, detail = pin()
    assert ok, detail


MUTANTS = {
    1: "Sturm recurrence uses e instead of e^2",
    2: "sign error in the LU elimination of T - lambda I",
    3: "no Gram-Schmidt inside groups",
    4: "double-double product drops a cross term",
    5: "a zero pivot of the Sturm count counted as negative (count at sigma + 0)",
    6: "a zero pivot of the elimination left unguarded",
    7: "||T||_1 without the right off-diagonal of each row",
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS), ids=lambda m: MUTANTS[m])
def test_pins_reject_mutant(mutant, tmp_path):
    """Each planted mistake in the oracle must make at least one pin fail."""
    path = oracle.build(out=os.path.join(str(tmp_path), f"liboracle_m{mutant}.so"), mutant=mutant)
    try:
        oracle.use_library(path)
        failed = []
        for pin in P.ALL_PINS:
            try:
                ok, _ = pin()
            except Exception:  # a crash in a pin also counts as a rejection
                ok = False
            if not ok:
                failed.append(pin.__name__)
                break
        assert failed, f"mutant {mutant} ({MUTANTS[mutant]}) passed every pin"
    finally:
        oracle.use_library(None)
