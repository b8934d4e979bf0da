"""Tolerances shared by the GPU parity tests."""

U_FP32 = 2.0 ** -24   # unit roundoff of IEEE single precision


def mixed_forward_bound(eps: float) -> float:
    """Bound on ||x_mixed - x_oracle|| / ||x_oracle|| for the FP32 factor and solve
    before refinement, against the FP64 oracle at the same eps: the truncation part
    (10 eps, as for the FP64 form) plus the FP32 rounding part, GROWTH * u_32.  Every
    stored entry carries a relative rounding of u_32 and a solve applies about
    2 log2(n) HODLR blocks in sequence; GROWTH = 100 allows that count (20 at
    n = 1024) times a factor 5 of amplification by the reduced blocks' conditioning.
    Measured: 9.4e-6 (64 x 64, leaf 16, eps 1e-6), 4.3e-7 (1024-wide strip, eps 1e-6),
    1.9e-7 (512-wide convection-diffusion strip, eps 1e-7)."""
    return 10.0 * eps + GROWTH * U_FP32


GROWTH = 100.0
