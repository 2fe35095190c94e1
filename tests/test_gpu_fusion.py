"""Step fusion: one launch per generation against objective + DE step as two
launches.  Two one-launch forms: the leading step (every workgroup repeats
the previous generation's DE step before its objective work; two buffer
slots alternate by launch parity) and the last-workgroup step (the DE step
in each block's last objective workgroup); the automatic choice picks one
of them by launch size.

Every form runs the same objective arithmetic, the same partial-sum
reduction (same thread count and order) and the same DE step, so fits must
be bit-identical: coefficients, objectives, flags, generations, final
populations and the best-so-far history.  Covered: the tiny block in both
precisions, the paper-scale block, a batch of uneven blocks sharing each
launch, the window stop rule with blocks stopping at different generations
(in both launch parities), a stop at generation 0 (value to reach), a
fit with no generation after the initial one, populations past one wave
(P = 100, 256), and fits with per-launch timing on (which run every form as
the objective alone plus the DE step).
"""
import numpy as np
import pytest

import synth
from gpu_util import block_of, ctx, settings_of, to_dev
from paper_1906_10598_amd import phasetrack as ptk

pytestmark = pytest.mark.gpu


FORMS = [ptk.PT_FUSION_LEAD, ptk.PT_FUSION_LAST, ptk.PT_FUSION_AUTO]


def _fit(mode, pbs, de):
    c = ctx()
    ptk.pt_ctx_set_step_fusion(c.handle, mode)
    try:
        fits = c.fit_batch(pbs, de) if len(pbs) > 1 else [c.fit_block(pbs[0], de)]
        pops = [ptk.pt_last_population(c.handle, k, de.pop) for k in range(len(pbs))]
        hists = [ptk.pt_last_history(c.handle, k, f.generations + 1) for k, f in enumerate(fits)]
    finally:
        ptk.pt_ctx_set_step_fusion(c.handle, ptk.PT_FUSION_AUTO)
    return fits, pops, hists


def _same(a, b, label):
    for k, (x, y) in enumerate(zip(a[0], b[0])):
        assert list(x.coef) == list(y.coef), (label, k)
        assert x.objective == y.objective and x.generations == y.generations and x.flags == y.flags
        assert np.array_equal(a[1][k][0], b[1][k][0]) and np.array_equal(a[1][k][1], b[1][k][1])
        assert np.array_equal(a[2][k], b[2][k])
    print(f"[{label}] {len(a[0])} block(s) bit-identical; generations {[f.generations for f in a[0]]}", flush=True)


@pytest.mark.parametrize("mode", FORMS)
@pytest.mark.parametrize("prec", [ptk.PT_PREC_FP64, ptk.PT_PREC_MIXED])
def test_tiny_block(prec, mode):
    b = synth.config0(1)
    dev = to_dev(b.samples)
    de = settings_of(b, precision=prec)
    _same(_fit(mode, [block_of(b, dev)], de), _fit(ptk.PT_FUSION_OFF, [block_of(b, dev)], de),
          f"fusion {mode} tiny {prec}")


@pytest.mark.parametrize("mode", FORMS)
def test_paper_block(mode):
    b = synth.config1(0)
    dev = to_dev(b.samples)
    de = settings_of(b)
    _same(_fit(mode, [block_of(b, dev)], de), _fit(ptk.PT_FUSION_OFF, [block_of(b, dev)], de),
          f"fusion {mode} paper")


@pytest.mark.parametrize("mode", FORMS)
def test_batch_with_window_rule(mode):
    blocks = synth.config3(1, nblocks=12, gens=400)
    devs = [to_dev(x.samples) for x in blocks]
    pbs = [block_of(x, d) for x, d in zip(blocks, devs)]
    de = settings_of(blocks[0], gens=400, rel_tol=1e-9, window=30)
    a, b = _fit(mode, pbs, de), _fit(ptk.PT_FUSION_OFF, pbs, de)
    gens = {f.generations for f in a[0]}
    assert len(gens) > 1  # blocks stopped at different generations
    assert len({g % 2 for g in gens}) == 2  # ... in both launch parities
    _same(a, b, f"fusion {mode} batch")


@pytest.mark.parametrize("mode", FORMS)
@pytest.mark.parametrize("window", [1, 2])
def test_short_windows(mode, window):
    # window 1 and 2: the rule compares with the step just stored / the one before
    b = synth.config0(2)
    dev = to_dev(b.samples)
    de = settings_of(b, gens=300, rel_tol=1e-3, window=window)
    a, o = _fit(mode, [block_of(b, dev)], de), _fit(ptk.PT_FUSION_OFF, [block_of(b, dev)], de)
    assert a[0][0].flags & ptk.PT_FLAG_CONVERGED
    _same(a, o, f"fusion {mode} window {window}")


@pytest.mark.parametrize("mode", FORMS)
def test_stop_at_generation_zero_and_no_generations(mode):
    b = synth.config0(3)
    dev = to_dev(b.samples)
    for de in (settings_of(b, vtr=1e9), settings_of(b, gens=0), settings_of(b, gens=1)):
        a, o = _fit(mode, [block_of(b, dev)], de), _fit(ptk.PT_FUSION_OFF, [block_of(b, dev)], de)
        assert a[0][0].generations == o[0][0].generations <= 1
        _same(a, o, f"fusion {mode} gens {de.max_gens} vtr {de.vtr}")


@pytest.mark.parametrize("mode", FORMS)
@pytest.mark.parametrize("pop", [100, 256])
def test_populations_past_one_wave(mode, pop):
    # P > 64: the leading step's selection spans several waves, its rows take
    # more than one round of loads (P > 73) and fewer threads sum each member's
    # partials (k = 256 / P); one block (arguments form) and a batch of two
    # (descriptor form), with a window stop
    b = synth.config0(4)
    dev = to_dev(b.samples)
    de = settings_of(b, gens=80, pop=pop, rel_tol=1e-6, window=10)
    _same(_fit(mode, [block_of(b, dev)], de), _fit(ptk.PT_FUSION_OFF, [block_of(b, dev)], de),
          f"fusion {mode} P {pop}")
    b2 = synth.config0(5)
    dev2 = to_dev(b2.samples)
    pbs = [block_of(b, dev), block_of(b2, dev2)]
    _same(_fit(mode, pbs, de), _fit(ptk.PT_FUSION_OFF, pbs, de), f"fusion {mode} P {pop} batch")


def test_invalid_fusion_mode():
    with pytest.raises(ptk.PtError):
        ptk.pt_ctx_set_step_fusion(ctx().handle, 4)


@pytest.mark.parametrize("mode", FORMS)
def test_timed_fit_equals_two_launch_form(mode):
    # with per-launch timing on, every form runs the objective alone and then
    # the DE step (events bracket the objective launches): the leading-step
    # instance must not be the one launched there
    b = synth.config1(0)
    dev = to_dev(b.samples)
    de = settings_of(b, gens=120)
    c = ctx()
    ptk.pt_ctx_set_timing(c.handle, True)
    try:
        a = _fit(mode, [block_of(b, dev)], de)
        nl, ms = ptk.pt_ctx_kernel_stats(c.handle)
    finally:
        ptk.pt_ctx_set_timing(c.handle, False)
    assert nl == de.max_gens + 1 and ms > 0.0
    _same(a, _fit(ptk.PT_FUSION_OFF, [block_of(b, dev)], de), f"timed fusion {mode} paper")


def test_graph_cache_eviction_keeps_fits_bitwise():
    # the leading-step form captures one graph per chunk (the launch index is
    # a kernel argument), of 50 generations when the window rule is on; a fit
    # of 13 000 generations needs 260 of them, more than a context caches
    # (256), so the cache evicts its least recently used quarter in the middle
    # of the fit (after waiting for the device, since the fit's earlier chunks
    # are still queued) and again during the next fit, which finds its first
    # chunks evicted.  (The window spans the whole fit, so the rule, on, never
    # stops it early.)
    b = synth.config0(2)
    dev = to_dev(b.samples)
    de = settings_of(b, gens=13_000, rel_tol=1e-300, window=13_000)
    with ptk.Context(0) as c:
        ptk.pt_ctx_set_step_fusion(c.handle, ptk.PT_FUSION_LEAD)
        first = c.fit_block(block_of(b, dev), de)
        second = c.fit_block(block_of(b, dev), de)
    ref = _fit(ptk.PT_FUSION_OFF, [block_of(b, dev)], de)[0][0]
    assert ref.generations == 13_000
    for f in (first, second):
        assert list(f.coef) == list(ref.coef) and f.objective == ref.objective
        assert f.generations == ref.generations and f.flags == ref.flags
    print(f"[graph eviction] 13000-generation fits bit-identical to the two-launch form", flush=True)
