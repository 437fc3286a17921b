"""Error models used by the GPU parity tests.

Worst case.  The recurrence v_{k+1} = 2 A_hat v_k - v_{k-1} evaluated in
precision u commits per step a local error delta_k with, row by row,
|delta_k| <= gamma u (2 |A_hat| |v_k| + |v_{k-1}|), gamma = (nnz per row + 2)
(the length of the FMA chain).  The error e_k = sum_i U_{k-i}(A_hat) delta_i
propagates through Chebyshev polynomials of the second kind, whose norm on a
spectrum inside [-1, 1] is at most k - i + 1, and |v_i| <= |z|.  Hence

    |mu_k^gpu - mu_k| <= |z|^2 gamma u (2 kappa + 1) k (k + 1) / 2 + dot terms,

kappa = max row sum of |A_hat|.  The symmetric ("doubling") form needs
k/2 steps for degree k and doubles the dot, giving a bound no larger.  This
bound is rigorous but grows with the row length: for dense rows (d entries)
it exceeds |mu_k| <= |z|^2 itself and pins nothing.

Random rounding model.  Following the probabilistic analysis of Higham and
Mary ("A new approach to probabilistic rounding error analysis", SIAM J. Sci.
Comput. 41(5), 2019), rounding errors are modelled as independent, mean-zero
random variables bounded by u times the rounded quantity.  Entry r of one
step 2 A_hat v = ca A v + cb v (ca = 2 alpha, cb = 2 beta) sums N products:
product errors contribute u_prod (sum_j A_rj^2 v_j^2)^(1/2) and the running
sum's roundings u_acc (sum_t s_t^2)^(1/2) <= u_acc sqrt(N) (max_t E s_t^2)^(1/2);
for probe-driven vectors (E[v v^T] = T_k(A_hat)^2, norm <= 1) both second
moments are at most rho^2, rho = the largest row 2-norm of A.  The epilogue
(scale, add, subtract, store) adds three roundings of magnitude <= u_acc
(ca rho + |cb| + 1).  So each local error entry has RMS at most

    sigma = ca (u_prod + u_acc sqrt(N)) rho + 3 u_acc (ca rho + |cb| + 1),

and, the entries being independent, z . U_m(A_hat) delta has RMS at most
sigma |U_m(A_hat) z| <= sigma (m + 1) |z|.  Summing the k independent steps,

    RMS(mu_k^gpu - mu_k) <= sigma |z| S(k),   S(k)^2 = sum_{m=1}^{k} m^2,

in the direct form; in the symmetric form mu_{2k} = 2 v_k.v_k - mu_0 and
mu_{2k+1} = 2 v_{k+1}.v_k - mu_1 carry at most 4 sigma |z| S(ceil(j / 2))
for degree j.  The tolerance is LAMBDA times that RMS where the worst-case
bound exceeds 1e-2 |z|^2 (``fp_moment_tol``).  This model has no
row-length factor beyond sqrt(N) and stays orders of magnitude below
|z|^2 for dense operators; ``tests/test_tolerance_controls.py`` checks on
the CPU that operators with a plausible kernel mistake (the lo part of a
split dropped, a row tile permuted, probe columns swapped) exceed it at the
tested shapes while faithful FP32 / BF16x3 emulations stay well inside.
"""
import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24
# BF16x3 product: each operand split as hi + lo with residual <= 2^-18
# relative (two round-to-nearest bf16 steps of 8 significant bits), and the
# dropped lo*lo term <= 2^-18 relative: at most 3 * 2^-18 per product.
U_BF16X3_PROD = 3.0 * 2.0 ** -18
# sigmas of the random-rounding model a tolerance spans
LAMBDA = 8.0


def kappa_csr(g, alpha, beta):
    """max_i sum_j |A_hat_ij| for A_hat = alpha*A + beta*I."""
    A = g.to_scipy()
    A_hat = alpha * A
    A_hat.setdiag(A_hat.diagonal() + beta)
    return float(np.max(np.abs(A_hat).sum(axis=1)))


def rho_rows(A):
    """Largest row 2-norm of A (dense ndarray or scipy.sparse)."""
    if hasattr(A, "multiply"):
        return float(np.sqrt(np.max(np.asarray(A.multiply(A).sum(axis=1)))))
    A = np.asarray(A, dtype=np.float64)
    return float(np.max(np.sqrt(np.einsum("ij,ij->i", A, A))))


def moment_tol(n, mu0, u, row_nnz, kappa):
    """Worst-case per-degree absolute tolerance array [n+1]."""
    k = np.arange(n + 1, dtype=np.float64)
    gamma = row_nnz + 2
    rec = mu0 * gamma * u * (2 * kappa + 1) * k * (k + 1) / 2
    dots = 4 * mu0 * U64 * mu0 + 1e-300  # FP64 accumulation of exact products
    return rec + dots


def moment_rms(n, z2, u_prod, u_acc, n_acc, rho, alpha, beta, doubling=False):
    """Random-rounding model: per-degree RMS of mu_j^gpu - mu_j, array [n+1]."""
    ca, cb = 2.0 * abs(alpha), 2.0 * abs(beta)
    sigma = ca * (u_prod + u_acc * np.sqrt(n_acc)) * rho + 3.0 * u_acc * (ca * rho + cb + 1.0)
    j = np.arange(n + 1, dtype=np.float64)

    def S(k):
        return np.sqrt(k * (k + 1) * (2 * k + 1) / 6.0)

    if doubling:
        return 4.0 * sigma * np.sqrt(z2) * S(np.ceil(j / 2))
    return sigma * np.sqrt(z2) * S(j)


def fp_moment_tol(n, z2, prec, n_acc, rho, kappa, alpha, beta, doubling=False):
    """Tolerance [n+1] for FP32 ("fp32") or BF16x3 ("bf16x3") moments.  Per
    degree: the rigorous worst-case bound wherever it pins the result (below
    1e-2 |z|^2, as for short stencil rows), else LAMBDA times the
    random-rounding RMS (dense and long rows), plus the FP64 accumulation of
    the moment dots.  The random model is not used where the rigorous bound
    suffices because the roundings of a constant-coefficient stencil are not
    independent: on the 2D Laplacian 2048^2 the FP32 errors reach 2.5 times
    the model's 8-sigma bound (yet only 8e-8 |z|^2)."""
    u_prod = U32 if prec == "fp32" else U_BF16X3_PROD
    u_worst = U32 if prec == "fp32" else 2.0 ** -16
    worst = moment_tol(n, z2, u_worst, n_acc, kappa)
    model = LAMBDA * moment_rms(n, z2, u_prod, U32, n_acc, rho, alpha, beta, doubling)
    model = np.minimum(worst, model + 4 * z2 * U64 * z2 + 1e-300)
    return np.where(worst <= 1e-2 * z2, worst, model)


def learned_g_tol(mu, c, F, aff, P):
    """Per-probe bounds on |g_gpu - g| for the learned level's inference,
    g the oracle's ``composite_g`` with bfloat16 roundings.

    Returns (tight, loose).  Both sides round the same quantities to bf16,
    but their pre-rounding values differ by FP32 versus FP64 accumulation
    and tanhf versus tanh, so a value lying within that difference of a
    rounding boundary can round to the neighbouring bf16 number (one unit in
    the last place, at most 2^-7 relative).  ``loose`` bounds the output to
    first order when any number of such roundings differ (tanh is
    1-Lipschitz); ``tight`` assumes none does (FP32 accumulation and tanhf
    error only).  Both add the affine stages' parity (beta to 2e-6, ybar and
    ysd to 1e-8 relative, FP64 moments)."""
    from oracle import mlp as omlp

    mu = np.asarray(mu, dtype=np.float64)
    r = omlp.bf16_round
    u = omlp.standardized(mu[:, :F] / mu[:, :1], aff.xmean[:F], aff.xsd[:F])
    lin = np.abs(u) @ np.abs(aff.lin[:F])
    h1s = r(np.tanh(r(u) @ r(P.W1).T + r(P.b1)))
    h2s = r(np.tanh(h1s @ r(P.W2).T + r(P.b2)))
    x, h1, h2 = np.abs(r(u)), np.abs(h1s), np.abs(h2s)
    W1, b1, W2, b2, w3 = (np.abs(r(a)) for a in (P.W1, P.b1, P.W2, P.b2, P.w3))
    b3 = abs(float(r(P.b3)))
    ulp, acc, th = 2.0 ** -7, U32, 4 * U32  # bf16 unit, FP32 rounding, tanhf error
    # no rounding differs: FP32 accumulation (F + 1 and H + 1 terms) and tanhf
    t_a1 = (F + 1) * acc * (x @ W1.T + b1)
    t_a2 = (t_a1 + th) @ W2.T + 65 * acc * (h1 @ W2.T + b2)
    t_out = (t_a2 + th) @ w3 + 65 * acc * (h2 @ w3 + b3)
    # any rounding may differ by one bf16 unit
    l_a1 = (ulp * x) @ W1.T + t_a1
    l_a2 = (l_a1 + ulp * h1 + th) @ W2.T + 65 * acc * (h1 @ W2.T + b2)
    l_out = (l_a2 + ulp * h2 + th) @ w3 + 65 * acc * (h2 @ w3 + b3)
    scale = mu[:, 0] * aff.ysd
    affine = (mu[:, 0] * (1e-8 * abs(aff.ybar) + 1e-12 * aff.ysd) + scale * 2e-6 * (1.0 + lin)
              + 1e-12 * np.abs(mu[:, :F]) @ np.abs(c[:F]) + 1e-10 * mu[:, 0])
    return scale * t_out + affine, scale * l_out + affine
