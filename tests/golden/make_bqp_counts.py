"""Writes bqp_counts.txt from the paper's printed closed forms (eq.
bqp-number-moments, eq. bqp-moment-number-constraints) via the oracle."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle.bqp import m_mom_closed_form, m_sos_closed_form  # noqa: E402

qs = list(range(1, 13)) + [20, 30, 40, 50, 60, 70, 80, 100, 120]
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "bqp_counts.txt"), "w") as f:
    f.write("# q n m_sos m_mom   (eq. bqp-number-moments, eq. bqp-moment-number-constraints)\n")
    for q in qs:
        n = 1 + q + q * (q - 1) // 2
        f.write(f"{q} {n} {m_sos_closed_form(q)} {m_mom_closed_form(q)}\n")
