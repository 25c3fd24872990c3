"""Algorithmic flop counts of IBMI, the numerators of the TFLOP/s figures.

Counts follow the paper's cost section: per set of b rows (c = p - b) the plan costs a
Cholesky factorisation (b^3/3), the inverse from it (2 b^3/3) and W = A_I^{-1} A_{I,I^c}
(2 b^2 c); each sweep costs the product W H_{I^c} (2 b c^2) and the diagonal update
V W^T (2 b^2 c) per set, plus 2 p^3 for the residual ||I - A H||_F.  They count what the
method computes, not what a kernel executes (the split forms run several products per
counted one).
"""


def plan_flops(p: int, ranges) -> float:
    tot = 0.0
    for s, e in ranges:
        b = e - s
        c = p - b
        tot += b ** 3 / 3.0 + 2.0 * b ** 3 / 3.0 + 2.0 * b * b * c
    return tot


def sweep_flops(p: int, ranges, with_residual: bool = True) -> float:
    tot = 0.0
    for s, e in ranges:
        b = e - s
        c = p - b
        tot += 2.0 * b * c * c + 2.0 * b * b * c
    if with_residual:
        tot += 2.0 * float(p) ** 3
    return tot
