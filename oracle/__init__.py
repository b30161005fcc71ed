"""CPU oracle for the matricized least-squares polynomial fit.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, links or runs anything in this package; only the
tests, the smoke check and the benchmark's CPU-baseline leg do.  The oracle
shares no code, header, table or helper with the HIP path.

What the method computes (Sec. II of the paper): given pairs (x_i, y_i),
i = 1..n, n >= 2, and a degree m, the coefficients a_0..a_m of
f(x) = a_0 + a_1 x + ... + a_m x^m that minimise Pi = sum_i [y_i - f(x_i)]^2
(Sec. II, the least-square-error objective and the polynomial model).  Setting
every dPi/da_j to zero gives the normal equations
sum_i x_i^j y_i = sum_k a_k sum_i x_i^(j+k), j = 0..m (Sec. II), i.e. A X = B
with the Hankel matrix A_jk = S_(j+k), S_p = sum_i x_i^p, and B_j = T_j =
sum_i x_i^j y_i; the paper solves it by Gaussian elimination (end of Sec. II).
In exact arithmetic this is the unique minimiser whenever the x_i take at
least m+1 distinct values, so the oracle is that minimiser computed as
accurately as plain code allows, three independent ways:

* ``fp64``     the paper's route in float64: power sums (correctly rounded
               with ``math.fsum``), Hankel assembly, Gaussian elimination with
               partial pivoting, optional affine change of variable.
* ``exact``    the same route in exact rational arithmetic (tiny inputs), plus
               exact power sums on a dyadic grid for large shifted inputs.
* ``qr``       the comparator of Sec. III: Householder QR of the Vandermonde
               matrix (and its tall-skinny tree form for large n).
* ``adjoint``  closed-form gradient of a loss of the coefficients with respect
               to every x_i and y_i, and central finite differences.
* ``c_oracle`` the float64 route in plain C (compensated sums, fixed chunk
               order, OpenMP over chunks), used for large inputs and timed as
               the CPU baseline.

Readings of the paper adopted here (the printed matrix A has A_00 = 1 and a
wrong last row; the derivative line drops the x_i^j factor; pivoting is not
specified) are stated where they are used.
"""
