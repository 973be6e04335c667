"""FP64 CPU oracle for Dual (O-)BDRS and its linear-memory certificate.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package: only the tests, the smoke check of the entry module and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
path; the only common module is the seeded input generator, which holds none
of the method's arithmetic.

Modules (each function cites the passage of the paper it follows):

* ``lse``          two-pass log-sum-exp over an implicit squared-Euclidean cost
* ``alg1``         Algorithm 1 (Dual O-BDRS, log domain), step by step
* ``certificate``  Proposition 3 and Algorithm 2 (log-domain upper bound)
* ``repair``       the feasible repair of the intermediate plan (proof of Prop. 3)
* ``primal``       primal-plan BDRS (Eq. 3), O-BDRS (Sec. 3.3) and IPOT with L
                   inner Sinkhorn steps, in the linear domain, dense, for pins
* ``lp``           exact LP optima used to bracket the certificate
* ``plan``         the state plan's marginals, marginal-error statistics and
                   barycentric projection (colour-transfer outputs)
* ``rounding``     two-sided rounding of the state plan onto Pi(r, c) (the
                   feasible-plan cost of the momentum / kernel ablation)

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against something other than itself (identities of the paper, exact LP
optima, closed forms, brute force).  No function is "parity unpinned".
"""
from . import lse, alg1, certificate, repair, primal, lp, plan, rounding  # noqa: F401
