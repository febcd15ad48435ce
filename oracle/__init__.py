"""CPU oracle for BLS12-377 G1 multi-scalar multiplication (test infrastructure).

This package is test infrastructure, not product code.  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it; the
GPU library never links, imports or calls anything here, and the oracle never
imports the GPU library.

Everything is plain CPython integer arithmetic, written for a reader who wants
to check it against the paper by eye:

* ``field``   -- curve constants derived from the BLS12 family parameter, the
                 base-field helpers, Montgomery-form conversion and a plain
                 word-by-word Montgomery reduction used to pin the lazy
                 reduction bounds.
* ``curve``   -- short-Weierstrass affine point addition (chord and tangent),
                 double-and-add scalar multiplication (Sec. II-D, curve
                 y^2 = x^3 + a x + b with a = 0, b = 1 for BLS12-377).
* ``te``      -- the twisted-Edwards form -x^2 + y^2 = 1 + (k/2) x^2 y^2 and
                 the extended coordinates (X, Y, T, Z), U = k T (Sec. II-D):
                 the birational map to and from the Weierstrass curve and
                 affine twisted-Edwards addition.
* ``msm``     -- the MSM definition sum_i s_i P_i and Pippenger's bucket
                 decomposition (Sec. II-C): digits, bucket sums, window sums,
                 group aggregation.
* ``points``  -- fixed-base generation of the synthetic point pools
                 P_i = k_i G used as test inputs.
"""
