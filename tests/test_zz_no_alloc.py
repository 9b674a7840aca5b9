"""lbib_adjoint_noalloc, the gradient call that allocates nothing (its
workspace is a static device array inside the library), against lbib_adjoint
with a caller-owned workspace: the same J and gradients on two calls in a row,
the second on a smaller lattice and run (the array keeps the first call's
contents), and a clear capacity error beyond the array's size."""
import numpy as np
import pytest

from paper_1903_03356_amd import lbib
from tests.parity import log
from tests.test_adjoint import ellipse_channel

pytestmark = pytest.mark.gpu


def _same(ref, got, rel):
    assert got["J"] == ref["J"]
    scale = max(abs(ref["dJ_dg"]), 1e-300)
    assert abs(got["dJ_dg"] - ref["dJ_dg"]) <= rel * scale, (got["dJ_dg"], ref["dJ_dg"])
    a, b = np.concatenate(ref["dJ_dks"]), np.concatenate(got["dJ_dks"])
    assert a.shape == b.shape
    assert np.max(np.abs(a - b)) <= rel * np.max(np.abs(a)), np.max(np.abs(a - b))


@pytest.mark.parametrize("real_bytes,mode,rel", [(8, "dynamic", 1e-10), (8, "kinematic", 1e-10),
                                                 (4, "dynamic", 1e-5)])
def test_noalloc_matches_workspace_call_twice(real_bytes, mode, rel):
    """First call: 64 x 40 channel, 32 nodes, 40 steps, whole tape.  Second
    call: 48 x 32 channel, 24 nodes, 25 steps, a checkpoint every 5 steps (a
    smaller workspace inside the same static array).  Each against
    lbib_adjoint on a fresh context of the same workload.  FP64 gradients agree
    to the rounding of the reverse kernel's atomics; FP32 ones to their own
    run-to-run spread."""
    big = ellipse_channel(real_bytes=real_bytes, mode=mode)
    small = ellipse_channel(real_bytes=real_bytes, mode=mode, nx=48, ny=32, n_nodes=24,
                            centre=(20.0, 13.0))
    cases = [(big, 40, 0, lbib.OBJ_TAYLOR), (small, 25, 5, lbib.OBJ_CENTROID_Y)]
    sizes = []
    for cfg, steps, every, obj in cases:
        ref = lbib.Sim(cfg).adjoint(steps, obj, 0, mode, checkpoint_every=every)
        sim = lbib.Sim(cfg)
        sizes.append(sim.adjoint_bytes(steps, every))
        got = sim.adjoint_noalloc(steps, obj, 0, mode, checkpoint_every=every)
        log(f"noalloc {cfg['nx']}x{cfg['ny']} {mode} rb{real_bytes}: J {got['J']!r} "
            f"dJ/dg {got['dJ_dg']:.6e} (workspace call {ref['dJ_dg']:.6e})")
        _same(ref, got, rel)
        assert sim.steps_done == steps
    assert sizes[1] < sizes[0] <= lbib.ADJOINT_SCRATCH_BYTES


def test_noalloc_rejects_oversize_workspace():
    """A 512 x 128 channel taped whole over 100 steps needs more than the
    static array holds: ECAPACITY with the sizes in the message, nothing run."""
    from paper_1903_03356_amd import workloads as wl
    cfg = wl.adjoint_channel()
    sim = lbib.Sim(cfg)
    need = sim.adjoint_bytes(100)
    assert need > lbib.ADJOINT_SCRATCH_BYTES
    with pytest.raises(lbib.LbibError) as e:
        sim.adjoint_noalloc(100)
    assert e.value.code == lbib.ECAPACITY
    assert str(need) in str(e.value)
    assert sim.steps_done == 0
    # the context is unchanged and still runs a gradient that fits (about 44 MB)
    assert sim.adjoint_bytes(10) <= lbib.ADJOINT_SCRATCH_BYTES
    got = sim.adjoint_noalloc(10)
    ref = lbib.Sim(cfg).adjoint(10)
    _same(ref, got, 1e-5)
