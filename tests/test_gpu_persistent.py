"""The persistent cooperative launch against the graph-replay launch.

Both launch strategies run the same objective arithmetic, the same
reduction order and the same DE step, so for a given geometry their fits
must be bit-identical: coefficients, objectives, final populations and the
best-so-far history.  Covered: one tiny block, the paper-scale block (the
workgroups keep their samples in registers), a batch of uneven blocks (more
work units than resident workgroups, samples re-read per unit), the window
stop rule (blocks stopping at different generations) and the mixed path.
"""
import numpy as np
import pytest

import synth
from gpu_util import block_of, ctx, settings_of, to_dev
from paper_1906_10598_amd import phasetrack as ptk

pytestmark = pytest.mark.gpu


def _fit(mode, pbs, de):
    c = ctx()
    ptk.pt_ctx_set_launch_mode(c.handle, mode)
    try:
        fits = c.fit_batch(pbs, de) if len(pbs) > 1 else [c.fit_block(pbs[0], de)]
        used = ptk.pt_ctx_last_launch(c.handle)
        pops = [ptk.pt_last_population(c.handle, k, de.pop) for k in range(len(pbs))]
        hists = [ptk.pt_last_history(c.handle, k, f.generations + 1) for k, f in enumerate(fits)]
    finally:
        ptk.pt_ctx_set_launch_mode(c.handle, ptk.PT_LAUNCH_AUTO)
    return fits, used, pops, hists


def _same(a, b, label):
    fa, ua, pa, ha = a
    fb, ub, pb, hb = b
    assert ua == ptk.PT_LAUNCH_PERSISTENT and ub == ptk.PT_LAUNCH_GRAPH, (ua, ub)
    for k, (x, y) in enumerate(zip(fa, fb)):
        assert list(x.coef) == list(y.coef), (label, k)
        assert x.objective == y.objective and x.generations == y.generations and x.flags == y.flags
        assert np.array_equal(pa[k][0], pb[k][0]) and np.array_equal(pa[k][1], pb[k][1])
        assert np.array_equal(ha[k], hb[k])
    print(f"[{label}] {len(fa)} block(s) bit-identical; generations {[f.generations for f in fa]}", flush=True)


@pytest.mark.parametrize("prec", [ptk.PT_PREC_FP64, ptk.PT_PREC_MIXED])
def test_tiny_block(prec):
    b = synth.config0(0)
    dev = to_dev(b.samples)
    de = settings_of(b, precision=prec)
    _same(_fit(ptk.PT_LAUNCH_PERSISTENT, [block_of(b, dev)], de),
          _fit(ptk.PT_LAUNCH_GRAPH, [block_of(b, dev)], de), f"tiny prec {prec}")


def test_paper_block_resident():
    b = synth.config1(0)
    dev = to_dev(b.samples)
    de = settings_of(b, gens=300)
    _same(_fit(ptk.PT_LAUNCH_PERSISTENT, [block_of(b, dev)], de),
          _fit(ptk.PT_LAUNCH_GRAPH, [block_of(b, dev)], de), "paper 300 gens")


def test_uneven_batch_streamed():
    # (some of these blocks fall outside the phasor bounds: the graph form
    # would run them apart with the per-sample arithmetic and the rest with
    # the phasor one, the persistent kernel all with the per-sample one, so
    # both sides are held to the per-sample arithmetic here)
    blocks = synth.config3(1, nblocks=12, gens=60)
    devs = [to_dev(b.samples) for b in blocks]
    pbs = [block_of(b, d) for b, d in zip(blocks, devs)]
    de = settings_of(blocks[0])
    c = ctx()
    ptk.pt_ctx_set_fp64_method(c.handle, ptk.PT_FP64_POLY)
    try:
        _same(_fit(ptk.PT_LAUNCH_PERSISTENT, pbs, de), _fit(ptk.PT_LAUNCH_GRAPH, pbs, de), "batch of 12")
    finally:
        ptk.pt_ctx_set_fp64_method(c.handle, ptk.PT_FP64_AUTO)


def test_window_rule_blocks_stop_at_different_generations():
    blocks = [synth.config0(s) for s in range(5)]
    devs = [to_dev(b.samples) for b in blocks]
    pbs = [block_of(b, d, stream=k) for k, (b, d) in enumerate(zip(blocks, devs))]
    de = settings_of(blocks[0], gens=2000, rel_tol=1e-9, window=25)
    a = _fit(ptk.PT_LAUNCH_PERSISTENT, pbs, de)
    _same(a, _fit(ptk.PT_LAUNCH_GRAPH, pbs, de), "window rule")
    gens = [f.generations for f in a[0]]
    assert all(f.flags & ptk.PT_FLAG_CONVERGED for f in a[0]) and len(set(gens)) > 1, gens
