"""pt_ctx_autotune (the batching pattern's tile / candidates-per-workgroup
tuner, Sec. 1.2's population parallelism): it returns a supported geometry,
caches it per (size class, P, precision), and a fit under the tuned geometry
is the fit with that geometry forced, bit for bit."""
import numpy as np
import pytest

import synth
from gpu_util import block_of, settings_of, to_dev
from paper_1906_10598_amd import phasetrack as ptk

pytestmark = pytest.mark.gpu

SPL = (4, 8, 16, 32)
CPG = (1, 2, 4, 8)


@pytest.mark.parametrize("precision", [ptk.PT_PREC_FP64, ptk.PT_PREC_MIXED])
def test_autotune_geometry_cache_and_bitwise_fit(precision):
    b = synth.config1(0)
    P = b.de.pop
    with ptk.Context(0) as c:  # a context of its own: tuning changes its geometry choices
        default = ptk.pt_ctx_get_tile(c.handle, b.n, P, precision)
        default_p1 = ptk.pt_ctx_get_tile(c.handle, b.n, P + 1, precision)
        default_small = ptk.pt_ctx_get_tile(c.handle, 1 << 17, P, precision)
        spl, cpg = ptk.pt_ctx_autotune(c.handle, b.n, P, precision, ptk.current_stream())
        print(f"[autotune prec={precision}] default {default} tuned {(spl, cpg)}", flush=True)
        assert spl in SPL and cpg in CPG
        # cached for the size class floor(log2 n), this P and precision only
        assert ptk.pt_ctx_get_tile(c.handle, b.n, P, precision) == (spl, cpg)
        assert ptk.pt_ctx_get_tile(c.handle, 300_000, P, precision) == (spl, cpg)  # 2^18 <= n < 2^19 as 400 000
        assert ptk.pt_ctx_get_tile(c.handle, 1 << 17, P, precision) == default_small  # other size class
        assert ptk.pt_ctx_get_tile(c.handle, b.n, P + 1, precision) == default_p1  # other population size
        # the tuned fit equals the fit with the tuned geometry forced
        dev = to_dev(b.samples)
        de = settings_of(b, gens=60, precision=precision)
        tuned = c.fit_block(block_of(b, dev), de)
        pop_t, f_t = ptk.pt_last_population(c.handle, 0, P)
        ptk.pt_ctx_set_tile(c.handle, spl, cpg)
        forced = c.fit_block(block_of(b, dev), de)
        pop_f, f_f = ptk.pt_last_population(c.handle, 0, P)
        ptk.pt_ctx_set_tile(c.handle, 0, 0)
        assert list(tuned.coef) == list(forced.coef) and tuned.objective == forced.objective
        assert np.array_equal(pop_t, pop_f) and np.array_equal(f_t, f_f)
        # a forced geometry wins over the tuned one; unsupported ones are refused
        ptk.pt_ctx_set_tile(c.handle, 8, 2)
        assert ptk.pt_ctx_get_tile(c.handle, b.n, P, precision) == (8, 2)
        ptk.pt_ctx_set_tile(c.handle, 0, 0)
        with pytest.raises(ptk.PtError):
            ptk.pt_ctx_set_tile(c.handle, 12, 4)
