"""Checkpoint and exact resume through the C ABI.

Every random number of the method is a pure function of the seed, the step,
the stream and the particle tags (Sec. 2.5), so a run split by a checkpoint
must equal the unbroken run bit for bit: a system saved at step k1 and
continued, and a fresh system set up with the same calls that loads the
checkpoint and runs the same steps, end with identical positions, image
counters, velocities, bonds, cumulative counters and last-sweep events.
"""

import numpy as np
import pytest

from paper_2609_21204_amd import dybond as db
from paper_2609_21204_amd import inputs
from test_gpu_modifiers import _melt_half_bound, _small
from test_gpu_parity import _assert_same_state, counters, log

pytestmark = pytest.mark.gpu


def _images(s):
    return s.positions(with_images=True)[1]


def _split_run(w, k1, k2, kt_source=db.DB_KT_SETPOINT, shape=None, batch_with=None):
    """Unbroken run of k1 + k2 steps against a checkpoint at k1 loaded into a
    new system (optionally with another step shape, or advanced inside a
    batch beside other systems)."""
    a = db.System.from_workload(w, kt_source=kt_source)
    b = db.System.from_workload(w, kt_source=kt_source)
    others = []
    try:
        if shape is not None:
            db.db_set_step_shape(b.h, *shape)
        a.step(k1)
        ck = a.save_checkpoint()
        a.step(k2)
        b.step(3)                       # a state of its own, replaced by the load
        b.load_checkpoint(ck)
        assert b.step_count == k1
        assert b.save_checkpoint() == ck, "a loaded state saves to the same bytes"
        ev, sk = b.sweep_events(db.DB_EVENT_FORMED)
        assert len(ev) == 0 and sk == db.NO_SWEEP
        if batch_with is None:
            b.step(k2)
        else:
            others = [db.System.from_workload(x) for x in batch_with]
            db.db_step_batch([b.h] + [o.h for o in others], k2)
        _assert_same_state(a, b, "resumed run")
        assert np.array_equal(_images(a), _images(b)), "image counters differ"
        return a.save_checkpoint(), counters(a)
    finally:
        for x in [a, b] + others:
            x.close()


@pytest.mark.parametrize("name,k1,k2,kt", [
    ("small", 137, 163, db.DB_KT_SETPOINT),
    ("small", 150, 150, db.DB_KT_KINETIC),
    ("telechelic", 140, 133, db.DB_KT_SETPOINT),
])
def test_resume_from_checkpoint_is_bit_identical(name, k1, k2, kt):
    """Checkpoints between two sweeps and right after one (k1 a multiple of
    the sweep period), in both temperature modes."""
    log(f"case checkpoint {name} at {k1} + {k2}, kT source {kt}")
    w = inputs.WORKLOADS[name](seed=3)
    _, c = _split_run(w, k1, k2, kt)
    assert c[:, 1].sum() > 0 and c[:, 2].sum() > 0
    log(f"checkpoint {name}: counters {c.tolist()}")


def test_resume_with_modifiers_and_another_step_shape():
    """Melting under the kinetic temperature and slip bonds (the full kernel
    variant), the loaded system running another launch shape."""
    log("case checkpoint with modifiers")
    _split_run(_small(5, melt=_melt_half_bound()), 93, 127, db.DB_KT_KINETIC, shape=(2, 0))
    _split_run(_small(6, bond=(db.DB_BOND_TETHER, 1.0, 0.5, 0.9, 1.1, 1.5), r_min=0.6, r_max=1.3, slip=2.0),
               61, 89, shape=(8, 0))


def test_resume_inside_a_batch():
    """The loaded system advanced by db_step_batch beside two others."""
    log("case checkpoint resumed in a batch")
    _split_run(inputs.small(seed=8), 121, 240, batch_with=[inputs.small(seed=9), inputs.telechelic(seed=9)])


def test_checkpoint_rejections_leave_the_state_alone():
    w = inputs.small(seed=2)
    log("case checkpoint rejections")
    with db.System.from_workload(w) as a, db.System.from_workload(w) as b:
        a.step(55)
        ck = a.save_checkpoint()
        size = db._U64()
        assert db.load().db_save_checkpoint(a.h, None, 0, db.ctypes.byref(size)) == db.DB_ETRUNC
        assert size.value == len(ck) == 48 + 24 + 36 * w.n + 12 * len(a.bonds())
        b.step(20)
        before = b.save_checkpoint()

        def status(data):
            try:
                b.load_checkpoint(data)
            except db.DybondError as e:
                return e.name
            return "DB_OK"

        bad = bytearray(ck)
        bad[100] ^= 1                                       # a payload byte
        assert status(bytes(bad)) == "DB_EINVAL"
        assert status(ck[:-4]) == "DB_EINVAL"               # truncated
        bad = bytearray(ck)
        bad[4] = 2                                          # format version
        assert status(bytes(bad)) == "DB_EINVAL"
        assert status(b"\0" * 48) == "DB_EINVAL"            # no magic
        assert b.save_checkpoint() == before, "a rejected load changed the state"
        w2 = inputs.small(seed=2)
        w2.seed = w.seed + 1                                # another random stream
        with db.System.from_workload(w2) as c:
            with pytest.raises(db.DybondError) as e:
                c.load_checkpoint(ck)
            assert e.value.name == "DB_EINVAL" and "set up differently" in str(e.value)
        b.load_checkpoint(ck)
        assert b.save_checkpoint() == ck


def test_resume_at_full_size_of_the_timed_gel():
    """The 200k gel of the benchmark: saved at an unaligned step after 1200
    steps (a renumbering and list builds behind it), resumed in a fresh
    system, 130 steps later bit-identical to the unbroken run."""
    w = inputs.gel(seed=1)
    log(f"case checkpoint gel n={w.n}")
    _, c = _split_run(w, 1237, 130)
    assert c[:, 1].sum() > 0


def test_resume_in_another_process(tmp_path):
    """A checkpoint written to a file and loaded by another process (its own
    HIP context and allocations) continues exactly as the unbroken run."""
    import os
    import subprocess
    import sys

    w = inputs.telechelic(seed=6)
    ck_file, out_file = tmp_path / "run.ckpt", tmp_path / "resumed.npz"
    log("case checkpoint across processes")
    with db.System.from_workload(w) as a:
        a.step(101)
        ck_file.write_bytes(a.save_checkpoint())
        a.step(99)
        ref = (a.positions(), a.velocities(), a.bonds(), counters(a))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    child = (
        "import sys, numpy as np\n"
        f"sys.path.insert(0, {root!r}); sys.path.insert(0, {os.path.join(root, 'tests')!r})\n"
        "from paper_2609_21204_amd import dybond as db, inputs\n"
        "from test_gpu_parity import counters\n"
        "w = inputs.telechelic(seed=6)\n"
        "with db.System.from_workload(w) as b:\n"
        f"    b.load_checkpoint(open({str(ck_file)!r}, 'rb').read())\n"
        "    b.step(99)\n"
        f"    np.savez({str(out_file)!r}, pos=b.positions(), vel=b.velocities(), bonds=b.bonds(), ctr=counters(b))\n"
    )
    r = subprocess.run([sys.executable, "-c", child], capture_output=True, text=True, timeout=150)
    assert r.returncode == 0, r.stderr[-2000:]
    got = np.load(out_file)
    for name, x, y in zip(("positions", "velocities", "bonds", "counters"), ref,
                          (got["pos"], got["vel"], got["bonds"], got["ctr"])):
        assert x.shape == y.shape and np.array_equal(x, y), f"{name} differ after resuming in another process"
