"""FP64 CPU oracle of the photon-package life cycle.

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library.
"""
from .oracle import (FLAG_ABSORB, FLAG_PEEL_EMIT, FLAG_PEEL_SCAT, FLAG_SPLIT, STAT_NAMES, detector_basis,
                     draw_words, dust_emission, emit_direction, emit_position, forced_tau, grad, grad_attached, hg_mu, hg_phase,
                     mbb_sum, peel, philox, reweight, rotate, run, trace, uniform)

__all__ = ["FLAG_ABSORB", "FLAG_PEEL_EMIT", "FLAG_PEEL_SCAT", "FLAG_SPLIT", "STAT_NAMES", "detector_basis",
           "draw_words", "dust_emission", "emit_direction", "emit_position", "forced_tau", "grad", "grad_attached", "hg_mu",
           "hg_phase", "mbb_sum", "peel", "philox", "reweight", "rotate", "run", "trace", "uniform"]
