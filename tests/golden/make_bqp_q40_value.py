"""Writes bqp_q40_seed0_value.txt: the optimal value of the order-2 moment
relaxation of the dense BQP q = 40, seed 0 (synth.bqp_instance), computed by
the FP64 oracle's Algorithm alg1 to eta_max <= 1e-8, together with the value
f(x) of the sign vector rounded from its rank-one solution (equal values
certify that the relaxation is tight and the value is the BQP minimum).
Takes a few minutes on a CPU."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import alm, bqp  # noqa: E402
from synth import bqp_instance, gaussian  # noqa: E402

q, seed = 40, 0
Q, c = bqp_instance(q, seed)
rel = bqp.build_relaxation(Q, c, "colex")
res = alm.solve(rel.cls, rel.counts, rel.b, gaussian(rel.n, 4, 100 + seed), alm.ALMOptions(p_max=128, n_neg=16))
x, fx = alm.rank_one_rounding(res.Y, Q, c, None)
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "bqp_q40_seed0_value.txt"), "w") as f:
    f.write("# dense BQP q=40 seed 0: oracle relaxation value, eta_max, rounded f(x) (written by make_bqp_q40_value.py)\n")
    f.write(f"value = {res.value!r}\n")
    f.write(f"eta_max = {max(res.eta)!r}\n")
    f.write(f"rounded = {fx!r}\n")
