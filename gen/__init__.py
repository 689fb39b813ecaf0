"""Seeded synthetic byte-stream generators and workload definitions.

This package produces the inputs that both the CPU oracle and the GPU library
are run on.  It holds none of the compression method's arithmetic: only
random-number generation, the synthetic sources that stand in for the paper's
datasets (Sec. 4.1, Table 1), and the plain-data description of each workload
(stream counts, lengths, model hyper-parameters).
"""

from .sources import (  # noqa: F401
    splitmix64,
    uniform01,
    markov_order2_table,
    markov2_streams,
    mixture_streams,
    zipf_pmf,
)
from .workloads import WORKLOADS, Workload, make_streams, truncate  # noqa: F401
