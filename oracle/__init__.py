"""CPU oracle for compressed modular matrix multiplication.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark may import, call, link or run anything in this
package.  It shares no code with the GPU library (no kernels, headers, helpers
or tables); the two only meet on the seeded inputs that the tests hand to both.

Contents
  reference  the plain definitions: the modular product (C library + a pure
             Python brute force), the Q-adic packings, digit extraction, REDQ,
             left and full compression (sections 4, 5) and ReduceAndCompress
             (procedure (1)).
  bounds     the paper's bounds relating p, k, Q = 2^t, d and the mantissa
             width, and the regime tests under which the floating-point
             accumulation is exact.
  emulate    a bit-exact emulation of the method's floating-point accumulation
             (integer arithmetic + round-to-nearest-even at beta bits), used to
             show that the bounds are tight.

Every function cites the passage of Dumas, Fousse and Salvy, "Compressed
Modular Matrix Multiplication" (2008) that it restates.
"""
