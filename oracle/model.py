"""The paper's performance model as closed forms (test infrastructure only).

Notation follows the paper's nomenclature table: d, r, t (fusion depth), K
(kernel points), D (bytes per element), C (flops), M (bytes), I = C / M,
PP (peak flop/s of a unit), BB (bandwidth, bytes/s), S (sparsity factor of a
transformation, fraction of non-zeros), alpha (fusion redundancy factor).

Equations (numbered by order of appearance in the paper):
  roofline            P = min(PP, BB * I)
  original problem    C = 2K, M = 2D, I = K / D
  CUDA-core fusion    I_CU(t) = t K / D, P_CU(t) = min(PP_CU, BB I_CU(t))
  redundancy          alpha = K(t) / (t K);  box: (2rt+1)^d / (t (2r+1)^d)
  tensor-core fusion  I_TC(t) = t (alpha / S) K / D,
                      P_TC,actual(t) = (S / alpha) min(PP_TC, BB I_TC(t))
  executed work       C_TC(t) = (alpha / S) C(t),  C(t) = t C
  speed-up ratio      P_TC,actual / P_CU,actual, four scenarios by which side
                      of its ridge each unit sits on
  sweet spot          (compute-bound on both) alpha < S PP_TC / PP_CU
  sparse units        I unchanged, PP_TC replaced by PP_SpTC

Star K and K(t) are not given in the paper; the reading used here is
K_star = 2dr+1 and K_star(t) = #{x : sum_i ceil(|x_i| / r) <= t}, the support
of the t-fold composed star.
"""
from __future__ import annotations

import itertools
import math


def K_points(shape: str, d: int, r: int) -> int:
    if shape == "box":
        return (2 * r + 1) ** d
    if shape == "star":
        return 2 * d * r + 1
    raise ValueError(shape)


def K_fused(shape: str, d: int, r: int, t: int) -> int:
    if shape == "box":
        return (2 * r * t + 1) ** d
    if shape == "star":
        R = r * t
        n = 0
        for x in itertools.product(range(-R, R + 1), repeat=d):
            if sum(math.ceil(abs(c) / r) for c in x) <= t:
                n += 1
        return n
    raise ValueError(shape)


def alpha(shape: str, d: int, r: int, t: int) -> float:
    return K_fused(shape, d, r, t) / (t * K_points(shape, d, r))


def alpha_box(d: int, r: int, t: int) -> float:
    return (2 * r * t + 1) ** d / (t * (2 * r + 1) ** d)


def flops_per_point(K: int) -> float:
    """C = 2K (one FMA = multiply + add per kernel point)."""
    return 2.0 * K


def bytes_per_point(D: float) -> float:
    """M = 2D (one read, one write)."""
    return 2.0 * D


def roofline(PP: float, BB: float, I: float) -> float:
    return min(PP, BB * I)


def I_cu(K: int, D: float, t: int) -> float:
    return t * K / D


def I_tc(K: int, D: float, t: int, a: float, S: float) -> float:
    return t * (a / S) * K / D


def C_tc(K: int, t: int, a: float, S: float) -> float:
    return (a / S) * t * 2.0 * K


def P_cu(PP_cu, BB, K, D, t):
    return roofline(PP_cu, BB, I_cu(K, D, t))


def P_tc_raw(PP_tc, BB, K, D, t, a, S):
    return roofline(PP_tc, BB, I_tc(K, D, t, a, S))


def P_tc_actual(PP_tc, BB, K, D, t, a, S):
    return (S / a) * P_tc_raw(PP_tc, BB, K, D, t, a, S)


def ridge(PP, BB):
    return PP / BB


def scenario(PP_cu, PP_tc, BB, K, D, t, a, S) -> int:
    """1: MB->MB, 2: MB->CB, 3: CB->MB, 4: CB->CB (CU side first)."""
    cu_cb = I_cu(K, D, t) > ridge(PP_cu, BB)
    tc_cb = I_tc(K, D, t, a, S) > ridge(PP_tc, BB)
    return {(False, False): 1, (False, True): 2, (True, False): 3, (True, True): 4}[(cu_cb, tc_cb)]


def speedup(PP_cu, PP_tc, BB, K, D, t, a, S) -> float:
    return P_tc_actual(PP_tc, BB, K, D, t, a, S) / P_cu(PP_cu, BB, K, D, t)


def sweet_spot(PP_cu, PP_tc, a, S) -> bool:
    return a < S * PP_tc / PP_cu


def gstencils(P_flops: float, K: int) -> float:
    """Point-steps per second / 1e9 at useful throughput P (flop/s)."""
    return P_flops / flops_per_point(K) / 1e9


def padding_utilisation(m_used: int, m_required: int) -> float:
    """Fraction of an MMA operand occupied by data when a dimension of size
    m_used is padded to m_required."""
    return m_used / m_required


def verdict(ratio: float, lo: float = 0.87, hi: float = 1.15) -> str:
    """'up', 'tie' or 'down' with a tie band on the ratio."""
    if ratio < lo:
        return "down"
    if ratio > hi:
        return "up"
    return "tie"
