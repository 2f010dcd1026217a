"""FP64 reference implementation of alternating-update NNCP (test oracle).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg, never by the GPU library or its binding.
It shares no code with the HIP path.

Everything is NumPy float64. Tensors are numpy arrays of shape
(I_1, ..., I_N); whatever their memory order, indices are logical, and the
matricisations below follow the paper's column-major convention (mode 1
fastest among the column modes, Section II-A and Section IV-C).

Readings of passages that are ambiguous or garbled in the paper are marked
"Reading:" where they are applied. Parity status: every function here is
pinned by a test under tests/ against brute force, a closed form, an
identity or an invariant, except where the docstring says "parity unpinned".
"""

from __future__ import annotations

import itertools
import math
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "unfold", "khatri_rao", "khatri_rao_list", "krp_for_mode",
    "mttkrp_bruteforce", "mttkrp_direct", "gram", "hadamard_others",
    "hals_update", "mu_update", "normalize_columns", "model_tensor_cp",
    "relerr_explicit", "fit_from_terms", "choose_split",
    "partial_mttkrp_left", "partial_mttkrp_right", "mttv_trail", "mttv_lead",
    "DimTree", "nncp", "nncp_unnormalized", "nnls_bruteforce", "contract_trailing", "contract_leading",
    "tree_split",
    "nls_objective", "kkt_residual", "MU_EPS", "subtree_schedule", "fit_of_model", "block_update",
]

MU_EPS = 1e-16


# ----------------------------------------------------------------------------
# Tensor notation (Section II-A)
# ----------------------------------------------------------------------------

def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n matricisation X_(n), an I_n x (I / I_n) matrix (Section II-A).

    Column index j = sum_{k != n} i_k * prod_{k' < k, k' != n} I_k', i.e. the
    remaining modes in increasing order with the lowest one fastest, which is
    the ordering that makes X_(n) K^(n) the MTTKRP with
    K^(n) = H^(N) (.) ... (.) H^(n+1) (.) H^(n-1) (.) ... (.) H^(1).
    """
    return np.moveaxis(np.asarray(X, dtype=np.float64), n, 0).reshape(X.shape[n], -1, order="F")


def khatri_rao(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Khatri-Rao product A (.) B, (I_A I_B) x R, column-wise Kronecker.

    Reading: the paper gives both a row-wise and a column-wise description
    (Section II-A) that disagree on which operand's index is fastest; the
    column-wise Kronecker form K(:,c) = A(:,c) kron B(:,c) is used, so the
    row of K with index j + I_B * i holds A(i,:) * B(j,:). With
    K^(n) = H^(N) (.) ... (.) H^(1) this makes H^(1)'s index fastest, which
    agrees with the column-major unfolding; brute force pins it.
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if A.shape[1] != B.shape[1]:
        raise ValueError("Khatri-Rao operands need the same column count")
    return (A[:, None, :] * B[None, :, :]).reshape(A.shape[0] * B.shape[0], A.shape[1])


def khatri_rao_list(mats: Sequence[np.ndarray]) -> np.ndarray:
    """mats[0] (.) mats[1] (.) ... (.) mats[-1] (left to right)."""
    K = np.asarray(mats[0], dtype=np.float64)
    for M in mats[1:]:
        K = khatri_rao(K, M)
    return K


def krp_for_mode(H: Sequence[np.ndarray], n: int) -> np.ndarray:
    """K^(n) = H^(N) (.) ... (.) H^(n+1) (.) H^(n-1) (.) ... (.) H^(1) (Section II-A)."""
    order = [H[k] for k in reversed(range(len(H))) if k != n]
    return khatri_rao_list(order)


# ----------------------------------------------------------------------------
# MTTKRP (Section II-A; element form written out in Section IV-A)
# ----------------------------------------------------------------------------

def mttkrp_bruteforce(X: np.ndarray, H: Sequence[np.ndarray], n: int) -> np.ndarray:
    """M^(n)(i, r) = sum over all other indices of X(i_1..i_N) prod_{k!=n} H^(k)(i_k, r).

    Plain loops over every tensor entry; for tiny tensors only.
    """
    X = np.asarray(X, dtype=np.float64)
    R = H[0].shape[1]
    M = np.zeros((X.shape[n], R))
    for idx in itertools.product(*[range(d) for d in X.shape]):
        x = X[idx]
        for r in range(R):
            p = x
            for k, ik in enumerate(idx):
                if k != n:
                    p *= H[k][ik, r]
            M[idx[n], r] += p
    return M


def mttkrp_direct(X: np.ndarray, H: Sequence[np.ndarray], n: int,
                  max_krp_rows: int = 1 << 21) -> np.ndarray:
    """M^(n) = X_(n) K^(n) with K^(n) formed explicitly (Section II-A).

    When K^(n) would be large, the columns of X_(n) are taken in blocks, one
    per index t of the slowest remaining mode `top`: those columns are
    contiguous in X_(n), and the matching rows of K^(n) are K_rest scaled
    by row t of H^(top) (K_rest = the Khatri-Rao product of the other
    remaining modes). Block t then contributes
    (X_(n)[:, block t] K_rest) * H^(top)(t, :); this is the same sum over
    columns, only split.
    """
    X = np.asarray(X)
    N = X.ndim
    R = H[0].shape[1]
    Xn = unfold(X, n)
    ncols = Xn.shape[1]
    if ncols <= max_krp_rows:
        return Xn @ krp_for_mode(H, n)
    top = max(k for k in range(N) if k != n)
    rest = [k for k in range(N) if k != n and k != top]
    K_rest = khatri_rao_list([H[k] for k in reversed(rest)]) if rest else np.ones((1, R))
    C = ncols // X.shape[top]
    Htop = np.asarray(H[top], dtype=np.float64)
    M = np.zeros((X.shape[n], R))
    for t in range(X.shape[top]):
        M += (Xn[:, t * C:(t + 1) * C] @ K_rest) * Htop[t][None, :]
    return M


# ----------------------------------------------------------------------------
# Gram matrices and their Hadamard product (Algorithm 1, lines with G and S)
# ----------------------------------------------------------------------------

def gram(H: np.ndarray) -> np.ndarray:
    """G = H^T H (R x R)."""
    H = np.asarray(H, dtype=np.float64)
    return H.T @ H


def hadamard_others(G: Sequence[np.ndarray], n: int) -> np.ndarray:
    """S^(n) = G^(1) * ... * G^(n-1) * G^(n+1) * ... * G^(N) (elementwise)."""
    R = G[0].shape[0]
    S = np.ones((R, R))
    for k, Gk in enumerate(G):
        if k != n:
            S = S * Gk
    return S


# ----------------------------------------------------------------------------
# NLS updates (Section II-B)
# ----------------------------------------------------------------------------

def hals_update(W: np.ndarray, S: np.ndarray, M: np.ndarray) -> np.ndarray:
    """One HALS sweep over the columns r = 1..R, in place (Gauss-Seidel).

    W(:,r) <- [ W(:,r) + (M(:,r) - (W S)(:,r)) / S(r,r) ]_+ using the
    already-updated columns r' < r.

    Reading: the paper prints the rule without the division by S(r,r)
    (Section II-B); that is the same rule when the other factors have unit
    columns (diag S = 1), which is how it is used after normalisation. The
    division keeps the step an exact coordinate minimiser for any scaling.
    Guard: S(r,r) = 0 (an all-zero column in another mode) sets column r
    to zero.
    """
    W = np.array(W, dtype=np.float64, copy=True)
    S = np.asarray(S, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    for r in range(W.shape[1]):
        srr = S[r, r]
        if not srr > 0.0:
            W[:, r] = 0.0
            continue
        W[:, r] = np.maximum(0.0, W[:, r] + (M[:, r] - W @ S[:, r]) / srr)
    return W


def mu_update(W: np.ndarray, S: np.ndarray, M: np.ndarray, eps: float = MU_EPS) -> np.ndarray:
    """Multiplicative update W <- W * M / max(W S, eps) (Lee-Seung rule).

    Reading: the paper names alternative NLS updates but does not print the
    multiplicative rule; the standard Lee-Seung form for the subproblem
    min_{W >= 0} 1/2 tr(W S W^T) - <M, W> is used.
    """
    W = np.asarray(W, dtype=np.float64)
    return W * np.asarray(M, dtype=np.float64) / np.maximum(W @ np.asarray(S, dtype=np.float64), eps)


def block_update(W: np.ndarray, S: np.ndarray, M: np.ndarray, update: str = "hals", sweeps: int = 1,
                 tol: float = 0.0) -> np.ndarray:
    """The NLS-Update of one block (Section II-B): the update rule applied
    `sweeps` times to the fixed subproblem min_{W >= 0} 1/2 tr(W S W^T) - <M, W>.

    Each row of W is a separate NNLS problem in its own unknowns. With tol > 0
    a row stops as soon as one application changes none of its entries by more
    than tol times its largest entry, so with a large `sweeps` every row is
    solved to that tolerance; for HALS (exact coordinate minimisation) that is
    the exact block solve the paper's faithful BCD asks for.
    """
    upd = {"hals": hals_update, "mu": mu_update}[update]
    W = np.array(W, dtype=np.float64, copy=True)
    M = np.asarray(M, dtype=np.float64)
    if tol <= 0.0:
        for _ in range(max(1, sweeps)):
            W = upd(W, S, M)
        return W
    active = np.arange(W.shape[0])
    for _ in range(max(1, sweeps)):
        if active.size == 0:
            break
        Wn = upd(W[active], S, M[active])
        change = np.max(np.abs(Wn - W[active]), axis=1)
        W[active] = Wn
        active = active[change > tol * np.max(np.abs(Wn), axis=1)]
    return W


def normalize_columns(W: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """lambda = column 2-norms of W, H = W diag(1/lambda) (appendix algorithm).

    A zero column stays zero and gets lambda_r = 0.
    """
    W = np.asarray(W, dtype=np.float64)
    lam = np.sqrt(np.sum(W * W, axis=0))
    inv = np.where(lam > 0, 1.0 / np.where(lam > 0, lam, 1.0), 0.0)
    return W * inv[None, :], lam


# ----------------------------------------------------------------------------
# Model, error and fit (Section IV-B; appendix algorithm)
# ----------------------------------------------------------------------------

def model_tensor_cp(lam: np.ndarray, H: Sequence[np.ndarray]) -> np.ndarray:
    """[[lambda; H^(1), ..., H^(N)]] = sum_r lambda_r H^(1)(:,r) o ... o H^(N)(:,r)."""
    dims = tuple(h.shape[0] for h in H)
    out = np.zeros(dims)
    for r in range(H[0].shape[1]):
        term = np.asarray(lam[r], dtype=np.float64)
        for h in H:
            term = np.multiply.outer(term, np.asarray(h[:, r], dtype=np.float64))
        out += term
    return out


def relerr_explicit(X: np.ndarray, lam: np.ndarray, H: Sequence[np.ndarray]) -> float:
    """||X - model|| / ||X|| formed entry by entry (small tensors only)."""
    X = np.asarray(X, dtype=np.float64)
    D = X - model_tensor_cp(lam, H)
    return math.sqrt(float(np.sum(D * D)) / float(np.sum(X * X)))


def fit_from_terms(alpha: float, beta: float, gamma: float) -> Tuple[float, float]:
    """epsilon = sqrt((alpha - 2 beta + gamma) / alpha), fit = 1 - epsilon.

    alpha = ||X||^2, beta = <X, model>, gamma = ||model||^2 (Section IV-B).
    Reading: the numerator is clamped at zero before the square root, since
    rounding can push it slightly negative when the model is exact.
    """
    num = max(0.0, alpha - 2.0 * beta + gamma)
    eps = math.sqrt(num / alpha) if alpha > 0 else 0.0
    return 1.0 - eps, eps


def fit_of_model(X: np.ndarray, lam: np.ndarray, H: Sequence[np.ndarray]) -> float:
    """fit = 1 - ||X - [[lam; H]]|| / ||X|| of a given model, for any tensor size.

    The error is expanded as in Section IV-B: ||X||^2 - 2 <X, model> + ||model||^2
    with <X, model> = sum_r lam_r (M^(1)(:, r) . H^(1)(:, r)), M^(1) the mode-1
    MTTKRP of X with the model's factors, and ||model||^2 = lam^T (*_n H^(n)T H^(n)) lam.
    Used to score a model found on one tensor (e.g. a 16-bit copy) against
    another (the FP32 original) without forming the model tensor.
    """
    X = np.asarray(X)
    lam = np.asarray(lam, dtype=np.float64)
    Hs = [np.asarray(h, dtype=np.float64) for h in H]
    Xf = X.reshape(-1, order="A")
    alpha = float(np.dot(Xf.astype(np.float64, copy=False), Xf.astype(np.float64, copy=False)))
    M1 = mttkrp_direct(X, Hs, 0)
    beta = float(np.sum(M1 * Hs[0], axis=0) @ lam)
    G = np.ones((lam.size, lam.size))
    for h in Hs:
        G = G * gram(h)
    gamma = float(lam @ G @ lam)
    return fit_from_terms(alpha, beta, gamma)[0]


# ----------------------------------------------------------------------------
# Dimension tree (Section IV-A, Figures 1 and 2)
# ----------------------------------------------------------------------------

def choose_split(dims: Sequence[int]) -> int:
    """Root split s (modes 1..s | s+1..N) minimising I_L + I_R.

    Reading: the paper asks for contiguous root splits and notes that the
    tree's temporary memory is smallest when the two halves have about
    equal size (Section IV-C, memory analysis); s is 1-based here and
    1 <= s <= N-1. Ties go to the smaller s.
    """
    dims = list(dims)
    best, best_cost = 1, None
    for s in range(1, len(dims)):
        cost = math.prod(dims[:s]) + math.prod(dims[s:])
        if best_cost is None or cost < best_cost:
            best, best_cost = s, cost
    return best


def partial_mttkrp_left(X: np.ndarray, H: Sequence[np.ndarray], s: int) -> np.ndarray:
    """Node {1..s}: T_L = X_[I_L x I_R] (H^(N) (.) ... (.) H^(s+1)), shape (I_1..I_s, R).

    X_[I_L x I_R] puts modes 1..s on the rows and is the tensor's own
    column-major layout (Section IV-A, Figure 2a).
    """
    dims = X.shape
    R = H[0].shape[1]
    IL = math.prod(dims[:s])
    Xm = np.asarray(X, dtype=np.float64).reshape(IL, -1, order="F")
    K = khatri_rao_list([H[k] for k in reversed(range(s, len(dims)))])
    return (Xm @ K).reshape(tuple(dims[:s]) + (R,), order="F")


def partial_mttkrp_right(X: np.ndarray, H: Sequence[np.ndarray], s: int) -> np.ndarray:
    """Node {s+1..N}: T_R = X_[I_L x I_R]^T (H^(s) (.) ... (.) H^(1)), shape (I_{s+1}..I_N, R)."""
    dims = X.shape
    R = H[0].shape[1]
    IL = math.prod(dims[:s])
    Xm = np.asarray(X, dtype=np.float64).reshape(IL, -1, order="F")
    K = khatri_rao_list([H[k] for k in reversed(range(0, s))])
    return (Xm.T @ K).reshape(tuple(dims[s:]) + (R,), order="F")


def mttv_trail(T: np.ndarray, H_rest: Sequence[np.ndarray]) -> np.ndarray:
    """Leaf {a} from node {a..b}: contract modes a+1..b of T (Figure 2b).

    T has shape (I_a, ..., I_b, R); for each r the leading I_a x J block of
    T(:, ..., :, r) (column-major) times column r of
    K = H^(b) (.) ... (.) H^(a+1) is one matrix-vector product.
    """
    Ia = T.shape[0]
    R = T.shape[-1]
    K = khatri_rao_list(list(reversed(list(H_rest))))
    T3 = np.asarray(T, dtype=np.float64).reshape(Ia, -1, R, order="F")
    return np.einsum("ijr,jr->ir", T3, K)


def mttv_lead(T: np.ndarray, H_a: np.ndarray) -> np.ndarray:
    """Node {a+1..b} from node {a..b}: contract mode a with H^(a) (Section IV-A)."""
    Ia = T.shape[0]
    R = T.shape[-1]
    T3 = np.asarray(T, dtype=np.float64).reshape(Ia, -1, R, order="F")
    out = np.einsum("ijr,ir->jr", T3, np.asarray(H_a, dtype=np.float64))
    return out.reshape(tuple(T.shape[1:-1]) + (R,), order="F")


def contract_trailing(T: np.ndarray, nkeep: int, H_rest: Sequence[np.ndarray]) -> np.ndarray:
    """Child {a..c} of node {a..b}: contract the last modes c+1..b of the node
    temporary T (shape (I_a, ..., I_b, R)) with their factors (Section IV-A):
    out(i, r) = sum_j T(i, j, r) K(j, r), i over the first `nkeep` modes and
    K = H^(b) (.) ... (.) H^(c+1) (H^(c+1)'s index fastest)."""
    R = T.shape[-1]
    keep = tuple(T.shape[:nkeep])
    K = khatri_rao_list(list(reversed([np.asarray(h, dtype=np.float64) for h in H_rest])))
    T3 = np.asarray(T, dtype=np.float64).reshape(math.prod(keep), -1, R, order="F")
    return np.einsum("ijr,jr->ir", T3, K).reshape(keep + (R,), order="F")


def contract_leading(T: np.ndarray, H_lead: Sequence[np.ndarray]) -> np.ndarray:
    """Child {c+1..b} of node {a..b}: contract the first modes a..c of T with
    their factors: out(j, r) = sum_i T(i, j, r) K(i, r), K = H^(c) (.) ... (.) H^(a)."""
    R = T.shape[-1]
    nlead = len(H_lead)
    rest = tuple(T.shape[nlead:-1])
    K = khatri_rao_list(list(reversed([np.asarray(h, dtype=np.float64) for h in H_lead])))
    T3 = np.asarray(T, dtype=np.float64).reshape(K.shape[0], -1, R, order="F")
    return np.einsum("ijr,ir->jr", T3, K).reshape(rest + (R,), order="F")


def tree_split(a: int, b: int, peel: int = 0) -> int:
    """Split point c of the internal node {a..b}: children {a..c} and {c+1..b}.

    Reading: the paper allows any binary tree over contiguous mode ranges
    (Section IV-A); its N = 5 example peels the first mode ({3,4,5} into
    {3} | {4,5}), the default here. Bit a*8 + b of `peel` (0-based modes)
    peels the last mode instead: {a..b-1} | {b}.
    """
    return b - 1 if (peel >> (a * 8 + b)) & 1 else a


def subtree_schedule(N: int, s: int, peel: int = 0) -> List[List[Tuple[str, Tuple[int, int], Optional[Tuple[int, int]]]]]:
    """The tree nodes computed just before each mode's update, in order.

    Reading: the root splits into {1..s} | {s+1..N} and every internal node by
    ``tree_split``. A node is computed immediately before its lowest mode is
    updated, from its parent: then modes below it are new and modes above it
    are old, which is what the direct MTTKRP of each of its leaves sees. A
    left child {a..c} of {a..b} contracts the parent's last modes (they are
    old); a right child {c+1..b} contracts its first modes a..c (new).
    Returns, for each mode n (0-based), a list of (kind, node, parent) with
    kind "pm_left" / "pm_right" (a root branch from the tensor, parent None),
    "trail" (left child) or "lead" (right child); nodes are (a, b) inclusive,
    and the last entry of mode n's list is its leaf (n, n).
    """
    out: List[List[Tuple[str, Tuple[int, int], Optional[Tuple[int, int]]]]] = []
    for n in range(N):
        lo, hi = (0, s - 1) if n < s else (s, N - 1)
        ops = []
        a, b, parent = lo, hi, None
        while True:
            if a == n:
                if parent is None:
                    ops.append(("pm_left" if lo == 0 else "pm_right", (a, b), None))
                else:
                    kind = "trail" if a == parent[0] else "lead"
                    ops.append((kind, (a, b), parent))
            if a == b:
                break
            c = tree_split(a, b, peel)
            parent = (a, b)
            a, b = (a, c) if n <= c else (c + 1, b)
        out.append(ops)
    return out


class DimTree:
    """Dimension-tree MTTKRP along a BCD sweep (Section IV-A).

    Call ``mttkrp(H, n)`` for n = 0, 1, ..., N-1 in order, updating H[n]
    between calls, exactly as Algorithm 1 does; nodes are computed by the
    validity rule in ``subtree_schedule``.
    """

    def __init__(self, X: np.ndarray, s: Optional[int] = None, peel: int = 0):
        self.X = np.asarray(X, dtype=np.float64)
        self.N = self.X.ndim
        self.s = choose_split(self.X.shape) if s is None else int(s)
        if not 1 <= self.s <= self.N - 1:
            raise ValueError("split must satisfy 1 <= s <= N-1")
        self.schedule = subtree_schedule(self.N, self.s, peel)
        self.node: Dict[Tuple[int, int], np.ndarray] = {}

    def mttkrp(self, H: Sequence[np.ndarray], n: int) -> np.ndarray:
        for kind, (a, b), parent in self.schedule[n]:
            if kind == "pm_left":
                T = partial_mttkrp_left(self.X, H, self.s)
            elif kind == "pm_right":
                T = partial_mttkrp_right(self.X, H, self.s)
            elif kind == "trail":
                T = contract_trailing(self.node[parent], b - a + 1, [H[k] for k in range(b + 1, parent[1] + 1)])
            else:
                T = contract_leading(self.node[parent], [H[k] for k in range(parent[0], a)])
            self.node[(a, b)] = T
        return self.node[(n, n)].reshape(self.X.shape[n], -1)


# ----------------------------------------------------------------------------
# BCD driver (Algorithm 1 with the appendix algorithm's normalisation and error)
# ----------------------------------------------------------------------------

def nncp(X: np.ndarray, H0: Sequence[np.ndarray], iters: int, update: str = "hals",
         lam0: Optional[np.ndarray] = None, mttkrp: str = "direct",
         split: Optional[int] = None, alpha: Optional[float] = None,
         callback: Optional[Callable[[int, int, dict], None]] = None,
         inner_sweeps: int = 1, inner_tol: float = 0.0, normalize: bool = True, peel: int = 0) -> dict:
    """Alternating-update NNCP, ``iters`` outer iterations (Algorithm 1).

    Each outer iteration visits the modes in order; for mode n it forms the
    MTTKRP M^(n), the Hadamard product S^(n) of the other modes' Grams, solves
    the block subproblem (``block_update``) and refreshes G^(n). With
    ``normalize`` (the appendix algorithm) the new block is split into unit
    columns and weights lambda; after the last mode the relative error comes
    from alpha = ||X||^2, beta = <M^(N), W^(N)> and
    gamma = lambda^T (S^(N) * G^(N)) lambda (Section IV-B).

    Readings:
    * all N factors are initialised by the caller (the paper initialises
      modes 2..N only, but HALS needs a starting H^(1)); with ``normalize``
      the starting factors are normalised first and their column norms are
      multiplied into lambda (``lam0`` defaults to ones);
    * the update for mode n starts from H^(n) diag(lambda) (the current
      model's mode-n block with the other factors at unit norm); the update
      rules are scale-covariant, so this equals the unnormalised iteration
      (``normalize=False``: plain factors, lambda fixed at ones) exactly;
    * fit = 1 - epsilon, recorded after every outer iteration;
    * ``inner_sweeps`` / ``inner_tol``: the block update applies the rule up
      to ``inner_sweeps`` times, row by row until a row stops changing
      (``block_update``). For HALS every sweep is an exact coordinate
      minimisation, so the sweeps converge to the exact NNLS solution that
      Section II-B names as the alternative to a single sweep (BPP solves it
      directly).

    ``mttkrp`` selects "direct" (the plain definition) or "tree" (the FP64
    dimension tree of root split ``split`` and internal splits ``peel``, used
    only to show that both give the same iterates).
    Returns dict(H=[...], lam=..., fit=[...], eps=[...]).
    """
    X = np.asarray(X)
    N = X.ndim
    R = H0[0].shape[1]
    lam = np.ones(R) if lam0 is None else np.array(lam0, dtype=np.float64)
    H = []
    for h in H0:
        if normalize:
            hn, nr = normalize_columns(h)
            H.append(hn)
            lam = lam * nr
        else:
            H.append(np.array(h, dtype=np.float64, copy=True))
    G = [gram(h) for h in H]
    if alpha is None:
        Xf = np.asarray(X, dtype=np.float64)
        alpha = float(np.sum(Xf * Xf))
    tree = DimTree(X, split, peel) if mttkrp == "tree" else None
    fits, epss = [], []
    for it in range(iters):
        M = S = W = None
        for n in range(N):
            M = tree.mttkrp(H, n) if tree is not None else mttkrp_direct(X, H, n)
            S = hadamard_others(G, n)
            start = H[n] * lam[None, :] if normalize else H[n]
            W = block_update(start, S, M, update, inner_sweeps, inner_tol)
            if normalize:
                H[n], lam = normalize_columns(W)
            else:
                H[n] = W
            G[n] = gram(H[n])
            if callback is not None:
                callback(it, n, dict(M=M, S=S, W=W, H=H, lam=lam))
        beta = float(np.sum(M * W))
        gamma = float(lam @ (S * G[N - 1]) @ lam)
        f, e = fit_from_terms(alpha, beta, gamma)
        fits.append(f)
        epss.append(e)
    return dict(H=H, lam=lam, fit=fits, eps=epss, alpha=alpha)


def nncp_unnormalized(X: np.ndarray, H0: Sequence[np.ndarray], iters: int,
                      update: str = "hals") -> List[np.ndarray]:
    """The factors of ``nncp`` run without normalisation (Algorithm 1 with plain
    factors); used to pin that the normalised iteration computes the same model."""
    return nncp(X, H0, iters, update=update, normalize=False)["H"]


# ----------------------------------------------------------------------------
# The NLS subproblem itself (Section II-B)
# ----------------------------------------------------------------------------

def nls_objective(W: np.ndarray, S: np.ndarray, M: np.ndarray) -> float:
    """1/2 tr(W S W^T) - <M, W>: the mode-n least-squares objective up to a constant.

    Reading: the paper prints the subproblem in normal-equation form; the
    problem it stands for is min_{W >= 0} ||X_(n) - W K^T||^2, which equals
    2 * (this) + ||X||^2 because K^T K = S and X_(n) K = M.
    """
    W = np.asarray(W, dtype=np.float64)
    return 0.5 * float(np.sum((W @ S) * W)) - float(np.sum(M * W))


def kkt_residual(W: np.ndarray, S: np.ndarray, M: np.ndarray) -> float:
    """Largest violation of W >= 0, grad >= 0, W * grad = 0 (grad = W S - M), relative."""
    W = np.asarray(W, dtype=np.float64)
    grad = W @ S - M
    scale = max(1e-300, float(np.max(np.abs(M))), float(np.max(np.abs(W @ S))))
    v1 = float(np.max(np.maximum(0.0, -W)))
    v2 = float(np.max(np.maximum(0.0, -grad))) / scale
    v3 = float(np.max(np.abs(W * grad))) / (scale * max(1e-300, float(np.max(np.abs(W))) or 1.0))
    return max(v1, v2, v3)


def nnls_bruteforce(S: np.ndarray, m: np.ndarray) -> np.ndarray:
    """Exact min_{h >= 0} 1/2 h^T S h - m^T h by enumerating active sets.

    For each subset F of {1..R} solve S_FF h_F = m_F with h = 0 off F and
    keep the KKT point (h_F >= 0, (S h - m)_i >= 0 off F). S must be
    symmetric positive definite; R should be small (2^R subsets).
    """
    S = np.asarray(S, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    R = S.shape[0]
    best, best_val = None, None
    for mask in range(1 << R):
        F = [i for i in range(R) if mask >> i & 1]
        h = np.zeros(R)
        if F:
            h[F] = np.linalg.solve(S[np.ix_(F, F)], m[F])
            if np.any(h[F] < -1e-14):
                continue
            h[F] = np.maximum(h[F], 0.0)
        g = S @ h - m
        off = [i for i in range(R) if i not in F]
        tol = 1e-10 * max(1.0, float(np.max(np.abs(m))))
        if off and np.any(g[off] < -tol):
            continue
        val = 0.5 * h @ S @ h - m @ h
        if best_val is None or val < best_val:
            best, best_val = h, val
    return best
