"""Seeded synthetic inputs for sampled sub-block hashing.

This package is the only code shared by the oracle side and the GPU side.  It
produces input bit blocks, Toeplitz seeds, explicit sampling assignments,
permutations and serving job streams.  It holds none of the method's
arithmetic: no sampling, no hashing, no concatenation.  Its random source is
numpy's PCG64, deliberately different from the SplitMix64 stream that the
method itself uses to draw the sampling variables V_i.
"""

from .gen import (  # noqa: F401
    WORD_BITS,
    n_words,
    bernoulli_bits,
    uniform_bits,
    permutation,
    assignment,
    unpack_bits,
    pack_bits,
)
from .configs import (  # noqa: F401
    CONFIGS, SERVING_P_BITS, TABLE1, TABLE1_N_SUB, config, serving_input,
    serving_input_device, serving_jobs, serving_planes, table1_instance)
