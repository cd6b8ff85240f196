"""FP64 CPU oracle for ManiDSDP (Wang, Hu, Xia, arXiv 2512.04406).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
package's smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does, and this package imports nothing from the product.

Everything is dense NumPy float64 and follows the paper's definitions:

* ``bqp``        order-2 moment relaxation of the binary quadratic program
                 (section "Why solve the dual formulation", paragraph on BQPs):
                 monomial basis, class map by symmetric difference, b, counts.
* ``operators``  A, A*, (AA*)^{-1}, the projectors P and Q
                 (eq. projection-operators), y(S) and D (section 3 opening).
* ``subproblem`` the reduced ALM subproblem cost (eq. reduced-ALM-subproblem),
                 its Euclidean gradient (Lemma lm:suboptimality), the oblique
                 manifold projector (Lemma sec4:lm1), Riemannian gradient and
                 Hessian (Proposition prop, eqs. sec4:eq6 / sec4:eq7) and the
                 row-normalisation retraction.
* ``rtr``        Riemannian trust region with truncated CG (Absil, Baker,
                 Gallivan 2007), the subproblem solver the paper uses.
* ``alm``        Algorithm alg1 (ManiDSDP) with the multiplier update, the
                 certificate X, the negative-curvature direction (Theorem
                 sec5:thm1), the sigma rule (eq. sec5:eq1) and the KKT
                 residuals of eq. res.
* ``brute``      exhaustive minimisation over {-1, 1}^q for tiny q.

Parity status of each function is recorded in its docstring.
"""
