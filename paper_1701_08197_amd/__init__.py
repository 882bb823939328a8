"""MI355X (gfx950) implementation of the LOFAR Online Flagger hot path
(van Nieuwpoort, arXiv 1701.08197): power, block median and stddev,
SumThreshold in time then frequency, SIR operator, history flagger, all in HIP
kernels behind the C ABI of include/lof.h."""
from . import _native  # noqa: F401
from ._native import (LOF_CI8, LOF_C64, LOF_F32, LOF_C64_AMP, LOF_OPT_AUTOCOMMIT,  # noqa: F401
                      LOF_OPT_LITERAL_HISTORY_TIE, LOF_OPT_GRAPH, LOF_OPT_PHASE_TIMING, LOF_OPT_SIR_PROSE,
                      LOF_OPT_INTEGRATED, LOF_OPT_ROBUST_SIGMA, LOF_OPT_PREFLAGGED, PHASES,
                      STATS_BYTES, LofTuning)
from .flagger import Block, Flagger, LofError, decode_stats, default_params, flag_blocks_static  # noqa: F401
