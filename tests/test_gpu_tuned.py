"""Held-out frames for every class of the tuned parameter table.

The tuner fits each class's parameters, its stop tolerance and its sweep
floor (min_sweeps) on four tuning images (workload seed 90: the four draws
of 16 with the widest holes). Here
every class solves a frame it was not tuned on (workload seed 97, at the
hard end of its density range: the fewest known pixels) with its table
entry, and the result must stay within the 0.5 grey-level bar of the
oracle's exact float64 solution in every channel, having run at least the
class's floor.
"""
import numpy as np
import pytest

import oracle
from paper_2110_03946_amd import autotune, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TABLE = autotune.load_table()
CLASSES = sorted(TABLE["classes"])


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def ddi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_03946_amd import ddi as mod
    mod.lib()
    return mod


@pytest.mark.parametrize("key", CLASSES)
def test_held_out_frame_per_class(ddi, key):
    size, kind, dens = key.split("/")
    h, w = (int(x) for x in size.split("x"))
    lo, _ = (float(x) for x in dens.split("-"))
    prm = TABLE["classes"][key]["params"]
    f, c = synth.make_workload(h, w, 3, lo, kind, workload=97, index=CLASSES.index(key))
    say("held-out", key, prm)
    with ddi.Plan(h, w, 3, **prm) as plan:
        u_t, st = plan.solve(torch.from_numpy(f).cuda(), torch.from_numpy(c).cuda())
    torch.cuda.synchronize()
    u = u_t.cpu().numpy()
    ex = oracle.solve_exact(f.astype(np.float64), c)
    err = np.abs(u - ex).reshape(3, -1).max(axis=1)
    say("  sweeps", st["sweeps"], "floor", prm["min_sweeps"], "err", err.round(3).tolist())
    assert st["converged"] == 1
    assert st["sweeps"] >= prm["min_sweeps"]
    assert err.max() <= 0.5, err
