"""The allocation-free sweep entry point (ddi_oras_sweep_noalloc) against
the allocating one (ddi_oras_sweep) through the C ABI.

Both run the same kernels on the same data, so the outputs and the float64
norms must agree bit for bit. Two calls in a row, the second on a smaller
image, check that the fixed scratch left behind by a larger call does not
leak into a smaller one; the size limit and the alias check are host-side
errors.
"""
import numpy as np
import pytest
import torch

from paper_2110_03946_amd import ddi, synth

pytestmark = pytest.mark.gpu


def _case(h, w, ch, seed):
    f, c = synth.make_workload(h, w, ch, 0.05, "bernoulli", workload=7, index=seed)
    rng = np.random.default_rng(seed)
    u0 = np.where(c[None] == 1, f, rng.uniform(0, 255, size=f.shape).astype(np.float32))
    return (torch.from_numpy(np.ascontiguousarray(u0, dtype=np.float32)).cuda(),
            torch.from_numpy(c).cuda())


# (h, w, channels, block, overlap, alpha, k): the two-wave 64-row sweep with a
# ragged last block column, then a smaller image on the single-wave path
SEQUENCE = [(300, 470, 3, 64, 4, 0.25, 6), (130, 70, 2, 32, 6, 0.5, 4)]


@pytest.mark.parametrize("order", [0, 1])
def test_noalloc_matches_allocating_sweep(order):
    seq = SEQUENCE if order == 0 else SEQUENCE[::-1] + SEQUENCE
    for i, (h, w, ch, S, o, al, k) in enumerate(seq):
        print(f"[noalloc] call {i}: {ch}x{h}x{w} S={S} o={o} k={k}", flush=True)
        u0, c = _case(h, w, ch, 11 + i)
        ref, rsq_ref = ddi.oras_sweep(u0, c, S, o, al, k)
        out = torch.full_like(u0, float("nan"))
        got, rsq = ddi.oras_sweep_noalloc(u0, c, S, o, al, k, u_out=out)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), f"call {i}: outputs differ"
        assert np.array_equal(rsq, rsq_ref), f"call {i}: norms {rsq} vs {rsq_ref}"


def test_noalloc_without_norms_and_errors():
    u0, c = _case(96, 160, 3, 5)
    ref, _ = ddi.oras_sweep(u0, c, 64, 4, 0.25, 8)
    got, none = ddi.oras_sweep_noalloc(u0, c, 64, 4, 0.25, 8, rsq=False)
    torch.cuda.synchronize()
    assert none is None and torch.equal(got, ref)
    # u_out overlapping u_in is rejected before any work
    with pytest.raises(ddi.DDIError) as e:
        ddi.oras_sweep_noalloc(u0, c, 64, 4, 0.25, 8, u_out=u0)
    assert e.value.code == ddi.DDI_EINVAL
    # an image whose transposed mask alone exceeds the fixed scratch
    h, w = 4160, 8192
    need = ddi.noalloc_scratch_bytes(h, w, 1, 64, 4)
    assert need > ddi.NOALLOC_SCRATCH_BYTES
    big = torch.zeros((1, h, w), dtype=torch.float32, device="cuda")
    cb = torch.ones((h, w), dtype=torch.uint8, device="cuda")
    with pytest.raises(ddi.DDIError) as e:
        ddi.oras_sweep_noalloc(big, cb, 64, 4, 0.25, 1)
    assert e.value.code == ddi.DDI_ESCRATCH
    # and the 4K RGB frame fits
    assert ddi.noalloc_scratch_bytes(2160, 3840, 3, 64, 4) <= ddi.NOALLOC_SCRATCH_BYTES
