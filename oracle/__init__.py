"""CPU FP64 oracle for the NEMD micro-solve, the Gaussian-process surrogate,
the MLP ensemble and the hybrid macro march.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import or call anything here.  The product
library (the HIP path) never does, and the oracle never imports it: the two
share no code.  The only module both sides use is ``workloads`` (seeded input
generators, no method arithmetic).

Modules
-------
md      ctypes wrapper over ``md_oracle.c`` (plain C, FP64, -ffp-contract=off)
gp      squared-exponential GP regression (numpy / scipy, FP64)
mlp     2-64-64-1 tanh ensemble with hand-written backward and Adam (numpy FP64)
hybrid  1-D mass-conservation march with surrogate queries and MD fallback
build   compiles ``md_oracle.c`` into ``libmd_oracle.so``
"""
