"""CPU reference for the LOF flagging path.  Test infrastructure only: imported by
tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg, never by the
product library."""
from .lof_oracle import *  # noqa: F401,F403
from .lof_oracle import Params, History, BlockResult, flag_block  # noqa: F401
