"""Automatic level selection (Section 3.2, Theorem thm:levels,
eqs. eqn:levelCost and eqn:costrecurrence).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 throughout.

From a pilot sample of per-probe terms t_j = c_j z^T T_j(A_hat) z
(an m_pilot x (n+1) table), the variance of a level variable
Q_{l'l} = sum_{j=l'+1}^{l} t_j (eq. def:qlevels) is the sample variance of
S_l - S_{l'} with prefix sums S_l = sum_{j<=l} t_j (S_{-1} = 0).  A sample
of Q_{l'l} costs C(l) = l matvecs (direct form) or ceil(l/2) (symmetric
form), Section 3.1.

The dynamic programme of Theorem thm:levels:
    Cbar_0 = 0,   Cbar_l = min_{0 <= l' < l} Cbar_{l'} + sqrt(V_{l'l} C(l)),
for 1 <= l <= n - 1.  The top level n is chosen with the extra condition of
Section 3.2: the sample size the allocation of eqs. eqn:optSamples /
eqn:optMu recommends for the highest level must be at least m_pilot.  For a
candidate second-highest level l' the total is T(l') = Cbar_{l'} +
sqrt(V_{l'n} C(n)) and that sample size is
    m_L = T(l') sqrt(V_{l'n} / C(n)) / eps^2        (target variance eps^2)
    m_L = B sqrt(V_{l'n} / C(n)) / T(l')              (budget B).
Readings (the paper leaves these open): the smallest l' wins ties; if no l'
meets the condition the single level {n} (l' = 0) is used; the j = 0 term is
part of the first level (l_0 = -1), which leaves its variance unchanged for
Rademacher probes since t_0 is the same for every probe; the recommended
sample sizes are rounded up and at least 2 (a level variance needs two
samples).

A plan may hold at most MAX_LEVELS levels (the fixed-size level arrays of
the library's interface).  When the optimum of the recurrence above has more,
the reading taken is the optimum over plans of at most MAX_LEVELS levels: the
same recurrence indexed by the number of levels,
    H_0(0) = 0, H_0(l > 0) = inf,
    H_k(0) = 0, H_k(l) = min_{0 <= l' < l} H_{k-1}(l') + sqrt(V_{l'l} C(l)),
so that H_k(l) is the least cost of at most k levels topped by l, and the
top level takes T(l') = H_{MAX_LEVELS - 1}(l') + sqrt(V_{l'n} C(n)) with the
same condition, ties and fallback.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

MAX_LEVELS = 32


def level_cost(l: int, doubling: bool) -> int:
    """Matvecs per sample of a level ending at degree l (Section 3.1)."""
    return (l + 1) // 2 if doubling else l


def level_variances(terms: np.ndarray) -> np.ndarray:
    """V[lp + 1, l] = sample variance (ddof 1) of sum_{j=lp+1}^{l} t_j over
    the pilot rows, for -1 <= lp < l <= n; other entries NaN."""
    terms = np.asarray(terms, dtype=np.float64)
    m, n1 = terms.shape
    S = np.cumsum(terms, axis=1)
    V = np.full((n1 + 1, n1), np.nan)
    for l in range(n1):
        V[0, l] = np.var(S[:, l], ddof=1)
        for lp in range(l):
            V[lp + 1, l] = np.var(S[:, l] - S[:, lp], ddof=1)
    return V


@dataclasses.dataclass
class Plan:
    degrees: list          # l_1 < ... < l_L = n
    m: list                # recommended samples per level (integers)
    var: list              # V_{l_{k-1} l_k} from the pilot
    cost: list             # C(l_k)
    m_real: list           # the real-valued allocation before rounding
    opt_total: float       # T(l') of the chosen second-highest level
    single_total: float    # sqrt(V_{0n} C(n)): the single level
    cbar: np.ndarray       # Cbar_0 .. Cbar_{n-1}


def _alloc(var, cost, target: float, budget: bool):
    s = sum(math.sqrt(v * c) for v, c in zip(var, cost))
    if s <= 0.0:
        return [0.0] * len(var)
    mu = (target / s) if budget else (s / target)
    return [mu * math.sqrt(v / c) if c > 0 else 0.0 for v, c in zip(var, cost)]


def _top(cbar, Vl, C, n, target, budget, m_pilot, single):
    """Second-highest level under the top-level condition (None: single)."""
    chosen, chosen_total = None, math.inf
    for lp in range(n):
        vt = max(Vl(lp, n), 0.0)
        tot = cbar[lp] + math.sqrt(vt * C[n])
        if not tot > 0.0:
            continue
        if budget:
            mL = target * math.sqrt(vt / C[n]) / tot
        else:
            mL = tot * math.sqrt(vt / C[n]) / target
        if mL >= m_pilot and tot < chosen_total:
            chosen, chosen_total = lp, tot
    if chosen is None:
        return 0, single
    return chosen, chosen_total


def select(V: np.ndarray, n: int, doubling: bool, target: float, budget: bool,
           m_pilot: int, max_levels: int = MAX_LEVELS) -> Plan:
    """Levels and sample sizes by the dynamic programme of Theorem thm:levels
    with the top-level condition of Section 3.2.  ``target`` is eps^2
    (budget = False) or the matvec budget B (budget = True).  Plans of more
    than ``max_levels`` levels are replaced by the best of at most that many
    (module docstring)."""
    C = [level_cost(l, doubling) for l in range(n + 1)]
    Vl = lambda lp, l: float(V[lp + 1, l])  # noqa: E731
    cbar = np.zeros(n)
    prev = np.zeros(n, dtype=np.int64)
    for l in range(1, n):
        best, arg = math.inf, 0
        for lp in range(l):
            v = cbar[lp] + math.sqrt(max(Vl(lp, l), 0.0) * C[l])
            if v < best:
                best, arg = v, lp
        cbar[l], prev[l] = best, arg
    single = math.sqrt(max(Vl(0, n), 0.0) * C[n])
    chosen, chosen_total = _top(cbar, Vl, C, n, target, budget, m_pilot, single)
    chain = [n]
    lp = chosen
    while lp > 0:
        chain.append(lp)
        lp = int(prev[lp])
    if len(chain) > max_levels:
        # H_k(l): at most k levels topped by l; H_k(0) = 0
        K = max_levels - 1
        H = np.full((K + 1, n), math.inf)
        H[:, 0] = 0.0
        prevk = np.zeros((K + 1, n), dtype=np.int64)
        for k in range(1, K + 1):
            for l in range(1, n):
                best, arg = math.inf, 0
                for lp in range(l):
                    if H[k - 1, lp] == math.inf:
                        continue
                    v = H[k - 1, lp] + math.sqrt(max(Vl(lp, l), 0.0) * C[l])
                    if v < best:
                        best, arg = v, lp
                H[k, l], prevk[k, l] = best, arg
        chosen, chosen_total = _top(H[K], Vl, C, n, target, budget, m_pilot, single)
        chain = [n]
        lp, k = chosen, K
        while lp > 0:
            chain.append(lp)
            lp, k = int(prevk[k, lp]), k - 1
    degrees = chain[::-1]
    lo = [0] + degrees[:-1]
    var = [max(Vl(a, b), 0.0) for a, b in zip(lo, degrees)]
    cost = [C[l] for l in degrees]
    mr = _alloc(var, cost, target, budget)
    m = [max(2, math.ceil(x)) for x in mr]
    return Plan(degrees, m, var, cost, mr, float(chosen_total), single, cbar)


def brute_cbar(V: np.ndarray, n: int, doubling: bool) -> np.ndarray:
    """Cbar_l of eq. eqn:levelCost by enumerating every level set
    0 < l_1 < ... < l_L = l (small n only): the minimum over all of them of
    sum_k sqrt(V_{l_{k-1} l_k} C(l_k)), with l_0 = 0; Cbar_0 = 0."""
    C = [level_cost(l, doubling) for l in range(n + 1)]
    out = np.zeros(n + 1)
    for l in range(1, n + 1):
        best = math.inf
        for r in range(0, l):
            for inner in itertools.combinations(range(1, l), r):
                degrees = list(inner) + [l]
                lo = [0] + degrees[:-1]
                tot = sum(math.sqrt(max(float(V[a + 1, b]), 0.0) * C[b]) for a, b in zip(lo, degrees))
                best = min(best, tot)
        out[l] = best
    return out


def brute_force_capped(V: np.ndarray, n: int, doubling: bool, target: float, budget: bool,
                       m_pilot: int, max_levels: int):
    """Every level set of at most max_levels levels topped by n (small n
    only): (least total, its degrees) among those meeting the top-level
    condition, else the single level."""
    C = [level_cost(l, doubling) for l in range(n + 1)]
    best, best_deg = math.inf, None
    for r in range(0, max_levels):
        for inner in itertools.combinations(range(1, n), r):
            degrees = list(inner) + [n]
            lo = [0] + degrees[:-1]
            tot = sum(math.sqrt(max(float(V[a + 1, b]), 0.0) * C[b]) for a, b in zip(lo, degrees))
            vt = max(float(V[lo[-1] + 1, n]), 0.0)
            if not tot > 0.0:
                continue
            mL = (target * math.sqrt(vt / C[n]) / tot if budget
                  else tot * math.sqrt(vt / C[n]) / target)
            if mL >= m_pilot and tot < best:
                best, best_deg = tot, degrees
    if best_deg is None:
        return math.sqrt(max(float(V[1, n]), 0.0) * C[n]), [n]
    return best, best_deg


def brute_force_budget(V: np.ndarray, n: int, doubling: bool, budget: float, m_pilot: int):
    """Budget form: every level set by enumeration; the least
    sum_k sqrt(V_k C_k) among those whose top level is recommended at least
    m_pilot samples (m_L = B sqrt(V_L / C_L) / total), else the single level.
    Returns the total."""
    C = [level_cost(l, doubling) for l in range(n + 1)]
    best = math.inf
    for r in range(0, n):
        for inner in itertools.combinations(range(1, n), r):
            degrees = list(inner) + [n]
            lo = [0] + degrees[:-1]
            tot = sum(math.sqrt(max(float(V[a + 1, b]), 0.0) * C[b]) for a, b in zip(lo, degrees))
            vt = max(float(V[lo[-1] + 1, n]), 0.0)
            if tot > 0.0 and budget * math.sqrt(vt / C[n]) / tot >= m_pilot:
                best = min(best, tot)
    return best if best < math.inf else math.sqrt(max(float(V[1, n]), 0.0) * C[n])
