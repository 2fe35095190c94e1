"""Step fusion: one launch per generation (the DE step in each block's last
objective workgroup) against objective + DE step as two launches.

The fused launch runs the same objective arithmetic, the same partial-sum
reduction (same thread count and order) and the same DE step, so fits must
be bit-identical: coefficients, objectives, flags, final populations and
the best-so-far history.  Covered: the tiny block in both precisions, the
paper-scale block, a batch of uneven blocks sharing each launch, and the
window stop rule with blocks stopping at different generations.
"""
import numpy as np
import pytest

import synth
from gpu_util import block_of, ctx, settings_of, to_dev
from paper_1906_10598_amd import phasetrack as ptk

pytestmark = pytest.mark.gpu


def _fit(fused, pbs, de):
    c = ctx()
    ptk.pt_ctx_set_step_fusion(c.handle, fused)
    try:
        fits = c.fit_batch(pbs, de) if len(pbs) > 1 else [c.fit_block(pbs[0], de)]
        pops = [ptk.pt_last_population(c.handle, k, de.pop) for k in range(len(pbs))]
        hists = [ptk.pt_last_history(c.handle, k, f.generations + 1) for k, f in enumerate(fits)]
    finally:
        ptk.pt_ctx_set_step_fusion(c.handle, True)
    return fits, pops, hists


def _same(a, b, label):
    for k, (x, y) in enumerate(zip(a[0], b[0])):
        assert list(x.coef) == list(y.coef), (label, k)
        assert x.objective == y.objective and x.generations == y.generations and x.flags == y.flags
        assert np.array_equal(a[1][k][0], b[1][k][0]) and np.array_equal(a[1][k][1], b[1][k][1])
        assert np.array_equal(a[2][k], b[2][k])
    print(f"[{label}] {len(a[0])} block(s) bit-identical; generations {[f.generations for f in a[0]]}", flush=True)


@pytest.mark.parametrize("prec", [ptk.PT_PREC_FP64, ptk.PT_PREC_MIXED])
def test_tiny_block(prec):
    b = synth.config0(1)
    dev = to_dev(b.samples)
    de = settings_of(b, precision=prec)
    _same(_fit(True, [block_of(b, dev)], de), _fit(False, [block_of(b, dev)], de), f"fused tiny {prec}")


def test_paper_block():
    b = synth.config1(0)
    dev = to_dev(b.samples)
    de = settings_of(b)
    _same(_fit(True, [block_of(b, dev)], de), _fit(False, [block_of(b, dev)], de), "fused paper")


def test_batch_with_window_rule():
    blocks = synth.config3(1, nblocks=12, gens=400)
    devs = [to_dev(x.samples) for x in blocks]
    pbs = [block_of(x, d) for x, d in zip(blocks, devs)]
    de = settings_of(blocks[0], gens=400, rel_tol=1e-9, window=30)
    a, b = _fit(True, pbs, de), _fit(False, pbs, de)
    assert len({f.generations for f in a[0]}) > 1  # blocks stopped at different generations
    _same(a, b, "fused batch")
