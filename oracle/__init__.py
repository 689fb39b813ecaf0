"""Plain, slow CPU oracle of the online-adaptive byte compressor.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the GPU
library; the two meet only through the seeded input generators.

What it computes (all floating point in FP64 unless stated):

* ``rng``        -- counter-based SplitMix64 initialisation of every weight
                    (no pretraining: encoder and decoder start from the same
                    random parameters, Sec. 2.1 "Overall Process").
* ``model``      -- the probability model: byte embedding, Latent
                    Transformation Engine (Sec. 3.2, Eqs. 14-16), a stack of
                    Multi-path Byte Refinement Blocks (Sec. 3.1.2, Eqs. 9-13),
                    output head and softmax giving Pr(i) (Eq. 1); the
                    cross-entropy loss (Eq. 2) and its hand-derived adjoint;
                    the Adam update (Sec. 4.1).
* ``quantize``   -- integer CDF from Pr(i); the decision is taken in FP32,
                    the precision of the GPU kernel.
* ``rangecoder`` -- multiply-first 32-bit range coder in exact Python
                    integers (the "Arithmetic Coding" step of Sec. 2.1).
* ``codec``      -- the autoregressive compression loop of Algorithm 1 run
                    over many streams in lockstep with one shared model.

Parity status of each function is listed in its module header.
"""

from .model import Config, Model  # noqa: F401
from .codec import encode, decode  # noqa: F401
