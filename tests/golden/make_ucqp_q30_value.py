"""Writes ucqp_q30_seed0_value.txt: the optimal value of the Hermitian order-2
moment relaxation of the UCQP q = 30, seed 0 (synth.ucqp_instance; real
embedding n = 992, m = 217,621 signed classes), computed by the FP64 oracle's
Algorithm alg1 to eta_max <= 1e-8, with the value z^H Q z of the unit-modulus
vector rounded from the moments M[e_i, 0] (equal values certify that the
relaxation is tight).  Takes several minutes on a CPU."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import alm, ucqp  # noqa: E402
from synth import gaussian, ucqp_instance  # noqa: E402

q, seed = 30, 0
Q = ucqp_instance(q, seed)
rel = ucqp.build_relaxation(Q)
res = alm.solve(rel.cls, rel.counts, rel.b, gaussian(rel.n, 8, 100 + seed), alm.ALMOptions(), w=rel.w)
z, fz = ucqp.rank_one_rounding(res.Y, Q)
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "ucqp_q30_seed0_value.txt"), "w") as f:
    f.write("# UCQP q=30 seed 0: oracle relaxation value, eta_max, rounded z^H Q z "
            "(written by make_ucqp_q30_value.py)\n")
    f.write(f"value = {res.value!r}\n")
    f.write(f"eta_max = {max(res.eta)!r}\n")
    f.write(f"rounded = {fz!r}\n")
    f.write(f"outer = {len(res.history)}\n")
