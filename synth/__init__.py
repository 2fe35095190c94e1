"""Seeded synthetic workloads shaped like the paper's open-loop tracking data.

This module only draws inputs (sample blocks, true coefficients, search
boxes, DE settings).  It holds none of the fit's arithmetic: no objective,
no DE, no observables.  Both the HIP path and the oracle take their inputs
from here; neither is imported.  ``synth.crlb`` gives the Cramer-Rao bounds
of the drawn blocks' parameters (Fisher information of the signal model), by
which the benchmark and the tests state f0 accuracy.

The paper's recordings (Mars Express, Chang'E-4 relay; Sec. 2.1, Sec. 4) are
not available, so these generators stand in for them with the paper's
shapes: real narrow-band samples quantised to 16 bit (Table 3), blocks of
hundreds of thousands of samples (Sec. 1.3, 400K per block), block lengths
up to 20 s (Sec. 4.1.1), and a cubic Taylor phase (Eq. 2-2-1, n = 3), or a
quartic one for perigee-like arcs (Sec. 3.2.1, n = 4).
"""
from .signals import (  # noqa: F401
    NSLOT,
    Block,
    DESettings,
    block_from_phase,
    config0,
    config1,
    config3,
    config4_stream,
    config_quartic,
    shift_truth,
    shift_truth4,
)
