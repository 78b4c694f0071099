"""Work model used to report throughput (Section 4.2's flop count).

The paper counts, for Algorithm 1 with d = n and q = 0: mn for Omega,
2mn^2 - n^2 for A^T Omega, 5n^3/3 for its QR, 2mn^2 - mn for A Qbar,
2mn^2 - n^3/3 for the QR giving Q, 2mn^2 - n^2 for Q^T A and 5n^3/3 for the
last QR (8mn^2 + 3n^3 - 2n^2 in all).  With d columns and q power rounds,
using the same conventions (2 r K c per product, 2 r d^2 - d^3/3 per QR of an
r x d panel):
  F = (2q+3) 2mnd + (q+2)(2nd^2 - d^3/3) + (q+1)(2md^2 - d^3/3).
"""

# MI355X peaks used for roofline fractions (dense, per GPU).
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0}
PEAK_HBM_GBS = 8000.0


def randqlp_flops(m, n, d, q):
    return ((2 * q + 3) * 2.0 * m * n * d + (q + 2) * (2.0 * n * d * d - d ** 3 / 3.0)
            + (q + 1) * (2.0 * m * d * d - d ** 3 / 3.0))


def passes_over_a(q):
    """Products that stream A: 2q + 3 (three at q = 0, as in Section 5.1)."""
    return 2 * q + 3
