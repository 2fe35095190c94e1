"""The serving loop (continuous batching with warm starts) on the GPU.

  * a block's result is the same alone and in the mix: every track's blocks
    fitted by a server that sees only that track equal, bit for bit, the
    results of a server that interleaves all tracks;
  * a served fit equals pt_fit_block on the same block with the box the
    server used (same kernels, same geometry), and its reported objective
    matches the FP64 oracle;
  * warm starts: the next block of a track starts from the previous fit
    re-expanded to its centre, in a box that holds the truth, and recovers f0;
  * admission under a tiny HBM budget still completes every block with the
    same results; a full queue answers PT_EBUSY.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_chi2_close, crlb_f0, ctx
from paper_1906_10598_amd import phasetrack as ptk

pytestmark = pytest.mark.gpu

GENS = 800


def _stream(ntracks=3, nblocks=8, seed=0):
    return synth.config4_stream(seed=seed, ntracks=ntracks, nblocks=nblocks, lengths=(100_000, 200_000))


def _settings():
    return ptk.make_settings(pop=40, max_gens=GENS, F=0.5, CR=0.9, seed=0x19061059 ^ 0xDE,
                             rel_tol=1e-9, window=50)


def _blk(item):
    b = item["block"]
    return ptk.make_block(__import__("torch").from_numpy(b.samples), b.fs, b.lo, b.hi, ref=b.ref,
                          stream=b.stream)


def _serve(items, budget=64 << 30, slots=16, gens_per_step=32, max_pending=4096):
    c = ctx()
    srv = ptk.pt_server_create(c.handle, ptk.make_server_config(
        _settings(), max_slots=slots, gens_per_step=gens_per_step, max_pending=max_pending,
        hbm_budget_bytes=budget))
    try:
        tickets = {}
        for it in items:
            t = ptk.pt_server_submit(srv, it["track"], _blk(it))
            assert t is not None
            tickets[t] = (it["track"], it["seq"])
        out = {}
        max_active = 0
        for _ in range(10000):
            a, p = ptk.pt_server_step(srv, ptk.current_stream())
            max_active = max(max_active, a)
            for r in ptk.pt_server_poll(srv):
                out[tickets[r.ticket]] = r
            if a == 0 and p == 0:
                break
        assert len(out) == len(items)
        return out, max_active
    finally:
        ptk.pt_server_destroy(srv)


def _key(r):
    return list(r.fit.coef) + [r.fit.objective, r.fit.generations, r.fit.flags]


def test_alone_equals_mix():
    items = _stream()
    mix, max_active = _serve(items)
    assert max_active >= 2  # blocks of several tracks really shared steps
    for tr in sorted({it["track"] for it in items}):
        alone, _ = _serve([it for it in items if it["track"] == tr])
        for k, r in alone.items():
            assert _key(r) == _key(mix[k]), k
    print(f"[server] {len(items)} blocks, up to {max_active} resident together; alone == mix", flush=True)


def test_served_fit_equals_fit_block_and_oracle():
    items = _stream(ntracks=2, nblocks=5, seed=1)
    res, _ = _serve(items)
    c = ctx()
    ptk.pt_ctx_set_tile(c.handle, 16, 4)
    try:
        for it in items:
            r = res[(it["track"], it["seq"])]
            b = it["block"]
            blk = _blk(it)
            blk.box = r.box
            f = c.fit_block(blk, _settings())
            assert list(f.coef) == list(r.fit.coef) and f.objective == r.fit.objective
            assert f.generations == r.fit.generations
            chi = oracle.chi2(b.samples.astype(np.float64), b.fs, b.ref, list(r.fit.coef))
            assert_chi2_close([r.fit.objective], [chi], b.n)
    finally:
        ptk.pt_ctx_set_tile(c.handle, 0, 0)


def test_warm_start_tracks_the_phase():
    items = _stream(ntracks=2, nblocks=8, seed=2)
    res, _ = _serve(items)
    cold, warm = [], []
    for it in items:
        r = res[(it["track"], it["seq"])]
        b = it["block"]
        err = abs(r.fit.coef[2] - b.truth[2])
        sig = crlb_f0(b)  # over the parameters the box frees (f0, f1 and f2 couple)
        print(f"[server warm] track {it['track']} seq {it['seq']} f0 err {err / sig:.2f} CRLB "
              f"gens {r.fit.generations}", flush=True)
        assert err < 12 * sig, (it["track"], it["seq"], err, sig)
        (warm if r.warm else cold).append(r.fit.generations)
        if r.warm:
            # the warm box is the cold half-width times 0.7 around the prediction
            w = (np.array(r.box.hi) - np.array(r.box.lo))[:5]
            assert np.allclose(w, 0.7 * (b.hi - b.lo)[:5], rtol=1e-12)
            assert r.box.lo[2] < b.truth[2] < r.box.hi[2]
    assert len(cold) == 2 and len(warm) == len(items) - 2
    # the window stop rule (1e-9 over 50 generations) dominates the generation
    # count, so a 0.7x box converges in about as many generations as a cold one
    print(f"[server warm] generations cold {cold} warm mean {np.mean(warm):.0f}", flush=True)


def _slot_bytes(n, spl=16, P=40):
    # bytes a resident block holds (pt_server_config.hbm_budget_bytes)
    ntiles = -(-n // (256 * spl))
    return n * 4 + (GENS + 1) * 8 + 2 * (P * 136 + P * ntiles * 8 + 48)


def test_tiny_budget_admits_one_at_a_time():
    items = _stream(ntracks=3, nblocks=5, seed=3)
    ref, _ = _serve(items)
    # room for one 200 000-sample block, not for two 100 000-sample ones
    assert _slot_bytes(200_000) < 2 * _slot_bytes(100_000)
    budget = (_slot_bytes(200_000) + 2 * _slot_bytes(100_000)) // 2
    small, max_active = _serve(items, budget=budget)
    assert max_active == 1
    for k in ref:
        assert _key(ref[k]) == _key(small[k])


def test_full_queue_is_busy():
    items = _stream(ntracks=1, nblocks=3, seed=4)
    c = ctx()
    srv = ptk.pt_server_create(c.handle, ptk.make_server_config(_settings(), max_pending=2))
    try:
        assert ptk.pt_server_submit(srv, 0, _blk(items[0])) is not None
        assert ptk.pt_server_submit(srv, 0, _blk(items[1])) is not None
        assert ptk.pt_server_submit(srv, 0, _blk(items[2])) is None
        assert ptk.pt_server_stats(srv)[1] == 2
    finally:
        ptk.pt_server_destroy(srv)


def test_leading_step_server_equals_default():
    # a server created under PT_FUSION_LEAD runs one leading-step launch per
    # generation (each block at its own launch index); its fits must equal
    # the default two-launch server's bit for bit
    items = _stream(ntracks=3, nblocks=6, seed=5)
    ref, _ = _serve(items)
    c = ctx()
    ptk.pt_ctx_set_step_fusion(c.handle, ptk.PT_FUSION_LEAD)
    try:
        lead, max_active = _serve(items)
    finally:
        ptk.pt_ctx_set_step_fusion(c.handle, ptk.PT_FUSION_AUTO)
    assert max_active >= 2
    for k in ref:
        assert _key(ref[k]) == _key(lead[k]), k


def test_served_stream_as_benchmarked():
    # The serving workload at full size: the first 32 arrivals of the 16-track
    # stream the benchmark serves (N in {1e5, 2e5, 4e5, 1e6} at 50 kHz), with
    # its settings (window 1e-9 over 50 generations, cap 3000; up to three
    # attempts with the range doubled; continuity limits 0.5 rad / 0.1 Hz),
    # submitted at once.  Sampled blocks -- the first of each length and every
    # retried one -- equal pt_fit_block in the box the server used, bit for
    # bit, and their objectives equal the oracle's chi^2 at their
    # coefficients; every block's f0 is within 12 Cramer-Rao bounds.
    items = synth.config4_stream(seed=0, ntracks=16, nblocks=160, rate=20.0)[:32]
    de = ptk.make_settings(pop=40, max_gens=3000, F=0.5, CR=0.9, seed=0x19061059 ^ 0xDE, rel_tol=1e-9, window=50)
    cfg = ptk.make_server_config(de, max_slots=64, gens_per_step=32, hbm_budget_bytes=64 << 30, max_attempts=3,
                                 enlarge=2.0, qc_phase_rad=0.5, qc_freq_hz=0.1)
    c = ctx()
    srv = ptk.pt_server_create(c.handle, cfg)
    try:
        tick = {}
        for k, it in enumerate(items):
            t = ptk.pt_server_submit(srv, it["track"], _blk(it))
            assert t is not None
            tick[t] = k
        res = {}
        for _ in range(100_000):
            a, p = ptk.pt_server_step(srv, ptk.current_stream())
            for r in ptk.pt_server_poll(srv):
                res[tick[r.ticket]] = r
            if a == 0 and p == 0:
                break
    finally:
        ptk.pt_server_destroy(srv)
    assert len(res) == len(items)
    lengths = sorted({it["block"].n for it in items})
    sample = sorted({min(k for k, it in enumerate(items) if it["block"].n == n) for n in lengths} |
                    {k for k, r in res.items() if r.attempts > 1})
    errs = []
    for k, it in enumerate(items):
        r, b = res[k], it["block"]
        assert not (r.fit.flags & ptk.PT_FLAG_ABANDONED), k
        errs.append(abs(r.fit.coef[2] - b.truth[2]) / crlb_f0(b))
    ptk.pt_ctx_set_tile(c.handle, 16, 4)  # the server's geometry
    try:
        for k in sample:
            r, b = res[k], items[k]["block"]
            blk = _blk(items[k])
            blk.box = r.box
            f = c.fit_block(blk, de)
            assert list(f.coef) == list(r.fit.coef) and f.objective == r.fit.objective, k
            assert f.generations == r.fit.generations, k
            chi = oracle.chi2(b.samples.astype(np.float64), b.fs, b.ref, list(r.fit.coef))
            assert abs(r.fit.objective - chi) <= 1e-10 * chi, (k, r.fit.objective, chi)
    finally:
        ptk.pt_ctx_set_tile(c.handle, 0, 0)
    print(f"[served stream] {len(items)} blocks, lengths {lengths}, sampled {sample} (retried "
          f"{sum(r.attempts > 1 for r in res.values())}): == pt_fit_block and the oracle's chi^2; f0 error median "
          f"{np.median(errs):.2f}, max {max(errs):.2f} CRLB", flush=True)
    assert max(errs) < 12.0
