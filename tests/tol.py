"""Error bounds shared by the GPU parity tests.

FP32 transfer blocks: the build inverts m - 1 plane Schur complements per
sweep (Gauss-Jordan on M x M blocks with FP32 products and an FP64 pivot
inverse) and chains them, so each block carries a relative error of order
eps32 sqrt(M) per elimination (the rounding of the M-term inner products
adds up like a random walk) and m of them along a sweep:
    max |S_gpu - S_oracle| / max |S_oracle|  <=  1.5 eps32 m sqrt(M).
Observed / bound (eps32 m sqrt(M) = 1): 0.15-0.55 over m = 2..32 and
M = 7..16129 (m = 16, M = 127: 2.4e-6; m = 32, M = 255: 9.6e-6; m = 4,
M = 191: 1.1e-6; m = 6, M = 529: 3.8e-6; m = 2, M = 7: 1.7e-7; full-size
m = 32, M = 1023 / 2047: 1.2e-5 / 1.3e-5; m = 8, M = 16129: 1.7e-5), so the
bound leaves a margin of 3-10x and a regression of that size fails.
"""
import math

EPS32 = 2.0 ** -24


def fp32_block_tol(m, M):
    return 1.5 * EPS32 * m * math.sqrt(M)
