"""CPU reference ("oracle") for the sparse-sketch library.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
implementation (no kernels, headers, helpers, tables or constant generators);
both sides take their inputs from the separate ``workloads`` generators, which
hold none of the method's arithmetic.

Everything here is plain and slow on purpose: FP64 (or exact integer /
rational) arithmetic, vectorised numpy where it is obviously equivalent to a
loop, and pure-Python loops for the tiny cases.  Each function cites the
passage of the paper ("Randomized Sketching is Robust to Low-Precision
Rounding on GPUs", Jeendgar, Flint, Anzt) or the external definition it
follows.

Modules
  philox    Philox4x32-10 counter-based generator (Salmon et al., SC'11).
  sketch    bucket/sign hash, explicit S, S@A in FP64, eta, mu, kappa.
  quant     FP32 -> FP16 round-to-nearest, exact stochastic rounding,
            dithered rounding, modelled exactly (integer / rational maths).
  model     what one sketch_apply call computes, including the per-unit
            FP32 partials and their FP16 quantisation and accumulation.
  ls        Householder least squares, LSQR, and the sketch-and-precondition
            iterative-refinement driver in FP64.
  native    ctypes front-end of the C FP64 oracle (liboracle.so), used for
            the full-size cases and for the CPU baseline timing.

Parity status of each function is listed in its docstring ("pinned by ...");
functions without an independent pin say "parity unpinned".
"""
