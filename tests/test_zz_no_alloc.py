"""The allocation-free bond read-out against the allocating one."""

import numpy as np
import pytest

from paper_2609_21204_amd import dybond as db
from paper_2609_21204_amd import inputs

pytestmark = pytest.mark.gpu


def test_noalloc_bond_readout_matches_db_read_bonds():
    """Two calls in a row on one device, the second with fewer bonds than the
    first (a stale tail of the shared staging array must not show), each
    equal to db_read_bonds bit for bit; a too-small buffer gives DB_ETRUNC
    with the count, as db_read_bonds does."""
    seen = []
    for name, steps in (("telechelic", 400), ("small", 60)):
        w = inputs.WORKLOADS[name](seed=3)
        with db.System.from_workload(w) as s:
            s.step(steps)
            ref = s.bonds()
            got = db.db_read_bonds_noalloc(s.h)
            print(f"{name}: {len(ref)} bonds", flush=True)
            assert len(ref) > 0
            assert got.shape == ref.shape and np.array_equal(got, ref)
            cnt = db._U64()
            st = db.load().db_read_bonds_noalloc(s.h, None, None, 0, db.ctypes.byref(cnt))
            assert st == db.DB_ETRUNC and cnt.value == len(ref)
            seen.append(len(ref))
    assert seen[1] < seen[0]
