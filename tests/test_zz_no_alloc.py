"""pt_objective_noalloc against pt_objective, through the C ABI.

The allocation-free entry point runs the same kernels in the library's fixed
device array instead of context buffers, so its objectives must equal
pt_objective's bit for bit.  Two calls in a row, the second smaller (fewer
samples and members), check that nothing of the first call's contents leaks
into the second; a call whose partial sums do not fit the array must be
rejected with a message and leave the next call correct.
"""
import numpy as np
import pytest

import synth
from gpu_util import block_of, ctx, random_population, to_dev
from paper_1906_10598_amd import phasetrack as ptk

pytestmark = pytest.mark.gpu


def _both(b, samples, pop, precision):
    import torch

    c = ctx()
    dev = to_dev(samples)
    blk = block_of(b, dev)
    p = to_dev(pop)
    want = c.objective(blk, p, precision).cpu().numpy()
    out = torch.full((pop.shape[0],), float("nan"), dtype=torch.float64, device="cuda")
    stream = ptk.current_stream()
    ptk.pt_objective_noalloc(c.handle, blk, p.data_ptr(), pop.shape[0], precision, out.data_ptr(), stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), want


@pytest.mark.parametrize("precision", [ptk.PT_PREC_FP64, ptk.PT_PREC_MIXED])
def test_noalloc_equals_pt_objective_twice_shrinking(precision):
    big = synth.config1(0)                   # 400 000 samples, P = 40
    small = synth.config1(1, n=50_000 + 77)  # ragged tail, P = 13
    rng = np.random.default_rng(7)
    for b, P in ((big, 40), (small, 13)):
        pop = random_population(rng, b.lo, b.hi, P, far=2)
        got, want = _both(b, b.samples, pop, precision)
        print(f"[noalloc n={b.n} P={P} prec={precision}] max |diff| {np.max(np.abs(got - want)):.3e}", flush=True)
        assert np.all(np.isfinite(got))
        np.testing.assert_array_equal(got, want)


def test_noalloc_rejects_oversize_then_works():
    import torch

    c = ctx()
    b = synth.config1(2, n=4096)
    pop = random_population(np.random.default_rng(3), b.lo, b.hi, 8)
    # a block whose partial sums exceed the array: P = 1024 members over
    # 2^23 samples need 1024 x 2048 x 8 bytes of partials at 16 samples per lane
    n_big = 1 << 23
    dev_big = torch.zeros(n_big, dtype=torch.float32, device="cuda")
    blk_big = ptk.make_block(dev_big, b.fs, b.lo, b.hi, stream=b.stream)
    pop_big = to_dev(random_population(np.random.default_rng(4), b.lo, b.hi, 1024))
    out_big = torch.empty(1024, dtype=torch.float64, device="cuda")
    with pytest.raises(ptk.PtError) as ei:
        ptk.pt_objective_noalloc(c.handle, blk_big, pop_big.data_ptr(), 1024, ptk.PT_PREC_FP64,
                                 out_big.data_ptr(), ptk.current_stream())
    assert ei.value.code == ptk.PT_EINVAL
    assert "bytes" in str(ei.value)
    # host samples are refused (the entry point stages nothing)
    blk_host = ptk.make_block(torch.from_numpy(b.samples), b.fs, b.lo, b.hi, stream=b.stream)
    with pytest.raises(ptk.PtError):
        ptk.pt_objective_noalloc(c.handle, blk_host, to_dev(pop).data_ptr(), 8, ptk.PT_PREC_FP64,
                                 out_big.data_ptr(), ptk.current_stream())
    got, want = _both(b, b.samples, pop, ptk.PT_PREC_FP64)
    np.testing.assert_array_equal(got, want)
