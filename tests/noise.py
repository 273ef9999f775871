"""Heuristic CKKS noise bounds in the slot domain (canonical embedding).

A random polynomial e with independent coefficients of variance V has slot
values with E|slot_j(e)|^2 = N V; products of polynomials multiply slot-wise.
Each bound takes 6 standard deviations for every random factor, so a product
term X*Y is bounded by (6 sd_X)(6 sd_Y).  h_s, h_v are Hamming weights of the
ternary secret and encryption randomness (about 2N/3)."""

import math

SIGMA = 3.2


def fresh(n, h_s, h_v, scale, sigma=SIGMA):
    """ENC noise e*v + e0 + e1*s (Sec. 3.4)."""
    g = 6 * sigma * math.sqrt(n)
    return g * (1 + 6 * math.sqrt(h_v) + 6 * math.sqrt(h_s)) / scale


def rescale_round(n, h_s, scale_after):
    """Rounding of both polynomials to integers after the exact division:
    eps0 + eps1*s with eps uniform in [-1/2, 1/2]."""
    g = 6 * math.sqrt(n / 12.0)
    return g * (1 + 6 * math.sqrt(h_s)) / scale_after


def key_switch(n, h_s, dnum, alpha_prod_max, n_digit, P, K, scale, sigma=SIGMA):
    """sum_j ext_j e_j / P (ext_j < n_digit * D_j as integers) plus the
    ModDown error eps0 + eps1*s with 0 <= eps < K + 1."""
    ext_sd = n_digit * alpha_prod_max / math.sqrt(3.0)
    t1 = dnum * (6 * ext_sd * math.sqrt(n)) * (6 * sigma * math.sqrt(n)) / P
    t2 = 6 * (K + 1) * math.sqrt(n) * (1 + 6 * math.sqrt(h_s))
    return (t1 + t2) / scale
