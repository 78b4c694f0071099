"""Flop model of Rand-QLP (Section 4.2), generalised to d columns and q rounds.

The paper itemises Algorithm 1 (d = n, q = 0) as: Omega mn; A^T Omega
2mn^2 - n^2; its QR 5n^3/3; A Qbar 2mn^2 - mn; the QR giving Q 2mn^2 - n^3/3;
Q^T A 2mn^2 - n^2; the final QR 5n^3/3; total 8mn^2 + 3n^3 - 2n^2.

Generalised, with the same conventions (a product r x K by K x c costs
2 r K c, a reduced QR of an r x d panel costs 2 r d^2 - d^3/3):
  F = (2q+3) * 2mnd + (q+2) * (2nd^2 - d^3/3) + (q+1) * (2md^2 - d^3/3).
At d = n, q = 0 this is 8mn^2 + 3n^3 + (lower order), i.e. the paper's total
up to its -2n^2 term.
"""


def randqlp_flops(m, n, d, q):
    gemm = (2 * q + 3) * 2.0 * m * n * d
    qr_n = (q + 2) * (2.0 * n * d * d - d ** 3 / 3.0)
    qr_m = (q + 1) * (2.0 * m * d * d - d ** 3 / 3.0)
    return gemm + qr_n + qr_m


def paper_flops_full(m, n):
    """The paper's printed total for Algorithm 1: 8mn^2 + 3n^3 - 2n^2."""
    return 8.0 * m * n * n + 3.0 * n ** 3 - 2.0 * n * n
