"""FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the GPU library and imports
nothing from it.  See pond_oracle.py for the method, its citations and the
readings taken where the paper is silent.
"""
from .pond_oracle import *  # noqa: F401,F403
from .pond_oracle import (DM_CONST_S, DM_CONST_TURNS, plan_geometry, n_blocks,  # noqa: F401
                          baseband_freqs_mhz, chirp_turns, ism_response,
                          dedispersion_chirp, unpack, dedisperse_block, dedisperse,
                          detect, decimate, fold_bins, fold, profiles_from, run,
                          disperse_pads, disperse, dispersion_delay_s,
                          residual_smear_ms, fft_length_eq1, search_geometry, search,
                          profile_snr)
