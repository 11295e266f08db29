"""Checks that pin an implementation of (F, F^T, H) to facts fixed by the paper
and by mathematics, independently of how the implementation computes.

Each check takes callables ``F(blocks, m)``, ``FT(blocks, d)``,
``H(blocks, m, noise_prec, prior_prec)`` working on FP64 numpy arrays
(time-outer layout, see the oracle) and returns the worst relative error it
saw.  They are used on the oracle (CPU) and, through small adapters, on the
GPU path.
"""
import numpy as np


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def dense_matrix(blocks):
    """Block (i, j) = F_{i-j} for i >= j, else 0 (eq. ShiftInvariance), assembled entry by entry."""
    Nt, Nd, Nm = blocks.shape
    A = np.zeros((Nt * Nd, Nt * Nm))
    for i in range(Nt):
        for j in range(i + 1):
            for s in range(Nd):
                for p in range(Nm):
                    A[i * Nd + s, j * Nm + p] = blocks[i - j, s, p]
    return A


def check_bruteforce(F, FT, rng, shapes):
    """Brute force on tiny shapes: compare with the assembled dense matrix."""
    worst = 0.0
    for (Nt, Nd, Nm) in shapes:
        blocks = rng.standard_normal((Nt, Nd, Nm))
        m = rng.standard_normal((Nt, Nm))
        d = rng.standard_normal((Nt, Nd))
        A = dense_matrix(blocks)
        worst = max(worst, rel(F(blocks, m), (A @ m.ravel()).reshape(Nt, Nd)))
        worst = max(worst, rel(FT(blocks, d), (A.T @ d.ravel()).reshape(Nt, Nm)))
    return worst


def lti_system(rng, Nu, Nd, Nm, Nt):
    """Random stable LTI system u_{k+1} = A u_k + C m_k, d = B u (section 2.1) and its blocks B A^k C."""
    A = rng.standard_normal((Nu, Nu))
    A *= 0.9 / max(abs(np.linalg.eigvals(A)))
    B = rng.standard_normal((Nd, Nu))
    C = rng.standard_normal((Nu, Nm))
    blocks = np.empty((Nt, Nd, Nm))
    Ak = np.eye(Nu)
    for k in range(Nt):
        blocks[k] = B @ Ak @ C
        Ak = A @ Ak
    return A, B, C, blocks


def check_lti(F, FT, rng, Nu=9, Nd=3, Nm=4, Nt=11):
    """F m equals time stepping the LTI system from u_0 = 0 (eq. LTI-time-discrete);
    F^T d equals the backward (adjoint) recursion lam_j = A^T lam_{j+1} + B^T d_j, (F^T d)_j = C^T lam_j."""
    A, B, C, blocks = lti_system(rng, Nu, Nd, Nm, Nt)
    m = rng.standard_normal((Nt, Nm))
    d = rng.standard_normal((Nt, Nd))
    u = np.zeros(Nu)
    dts = np.empty((Nt, Nd))
    for k in range(Nt):
        u = A @ u + C @ m[k]          # u_{k+1}
        dts[k] = B @ u                # paper's d_{k+1} is our output block k
    lam = np.zeros(Nu)
    mts = np.empty((Nt, Nm))
    for j in range(Nt - 1, -1, -1):
        lam = A.T @ lam + B.T @ d[j]
        mts[j] = C.T @ lam
    return max(rel(F(blocks, m), dts), rel(FT(blocks, d), mts))


def check_scalar_convolution(F, FT, rng, Nt=13):
    """Nd = Nm = 1: F is the lower-triangular Toeplitz matrix of a sequence, i.e. a truncated
    causal convolution (np.convolve); F^T is the correlation (convolution with the reversed input)."""
    f = rng.standard_normal(Nt)
    m = rng.standard_normal(Nt)
    d = rng.standard_normal(Nt)
    blocks = f.reshape(Nt, 1, 1)
    e1 = rel(F(blocks, m.reshape(Nt, 1)).ravel(), np.convolve(f, m)[:Nt])
    e2 = rel(FT(blocks, d.reshape(Nt, 1)).ravel(), np.convolve(f, d[::-1])[:Nt][::-1])
    return max(e1, e2)


def check_single_step(F, FT, rng, Nd=5, Nm=7):
    """Nt = 1: F is the single block F_0 (plain GEMV), F^T its transpose."""
    blocks = rng.standard_normal((1, Nd, Nm))
    m = rng.standard_normal((1, Nm))
    d = rng.standard_normal((1, Nd))
    return max(rel(F(blocks, m)[0], blocks[0] @ m[0]), rel(FT(blocks, d)[0], blocks[0].T @ d[0]))


def check_delta(F, FT, rng, Nt=6, Nd=3, Nm=4):
    """m = e_(j,p) gives (F m)_i = F_{i-j}[:, p] for i >= j and 0 before;
    d = e_(Nt-1,s) gives (F^T d)_j = F_{Nt-1-j}[s, :] (the last block row)."""
    blocks = rng.standard_normal((Nt, Nd, Nm))
    worst = 0.0
    for j in range(Nt):
        for p in range(Nm):
            m = np.zeros((Nt, Nm))
            m[j, p] = 1.0
            want = np.zeros((Nt, Nd))
            for i in range(j, Nt):
                want[i] = blocks[i - j][:, p]
            worst = max(worst, rel(F(blocks, m), want))
    for s in range(Nd):
        d = np.zeros((Nt, Nd))
        d[Nt - 1, s] = 1.0
        want = np.stack([blocks[Nt - 1 - j][s, :] for j in range(Nt)])
        worst = max(worst, rel(FT(blocks, d), want))
    return worst


def rank1_geometric(Nt, Nd, Nm, rho, rng):
    """F_k = rho^k u v^T; returns blocks, u, v."""
    u = rng.standard_normal(Nd)
    v = rng.standard_normal(Nm)
    blocks = (rho ** np.arange(Nt))[:, None, None] * np.outer(u, v)[None]
    return blocks, u, v


def closed_form_F(u, v, w, rho, Nt):
    """m_j = w for all j: (F m)_i = u (v.w) (1 - rho^{i+1}) / (1 - rho)."""
    i = np.arange(Nt)
    return ((1 - rho ** (i + 1)) / (1 - rho))[:, None] * (u * float(v @ w))[None, :]


def closed_form_FT(u, v, z, rho, Nt):
    """d_i = z for all i: (F^T d)_j = v (u.z) (1 - rho^{Nt-j}) / (1 - rho)."""
    j = np.arange(Nt)
    return ((1 - rho ** (Nt - j)) / (1 - rho))[:, None] * (v * float(u @ z))[None, :]


def check_closed_form(F, FT, rng, Nt=40, Nd=6, Nm=9, rho=0.93):
    blocks, u, v = rank1_geometric(Nt, Nd, Nm, rho, rng)
    w = rng.standard_normal(Nm)
    z = rng.standard_normal(Nd)
    m = np.tile(w, (Nt, 1))
    d = np.tile(z, (Nt, 1))
    return max(rel(F(blocks, m), closed_form_F(u, v, w, rho, Nt)),
               rel(FT(blocks, d), closed_form_FT(u, v, z, rho, Nt)))


def check_adjoint(F, FT, rng, Nt=17, Nd=5, Nm=11):
    """<F m, d> = <m, F^T d>; returned as |difference| / (|F m| |d|)."""
    blocks = rng.standard_normal((Nt, Nd, Nm))
    m = rng.standard_normal((Nt, Nm))
    d = rng.standard_normal((Nt, Nd))
    Fm = F(blocks, m)
    a = float(np.vdot(Fm, d))
    b = float(np.vdot(m, FT(blocks, d)))
    return abs(a - b) / (np.linalg.norm(Fm) * np.linalg.norm(d))


def check_hessian(H, rng, Nt=9, Nd=3, Nm=5, noise_prec=3.0, prior_prec=0.25):
    """H symmetric (<H m1, m2> = <m1, H m2>) and <m, H m> >= prior_prec |m|^2, and
    H equals noise_prec A^T A + prior_prec I of the dense matrix (brute force)."""
    blocks = rng.standard_normal((Nt, Nd, Nm))
    m1 = rng.standard_normal((Nt, Nm))
    m2 = rng.standard_normal((Nt, Nm))
    H1 = H(blocks, m1, noise_prec, prior_prec)
    H2 = H(blocks, m2, noise_prec, prior_prec)
    sym = abs(float(np.vdot(H1, m2)) - float(np.vdot(m1, H2))) / (np.linalg.norm(H1) * np.linalg.norm(m2))
    spd = 0.0 if float(np.vdot(m1, H1)) >= prior_prec * float(np.vdot(m1, m1)) else 1.0
    A = dense_matrix(blocks)
    Hd = noise_prec * A.T @ A + prior_prec * np.eye(A.shape[1])
    return max(sym, spd, rel(H1, (Hd @ m1.ravel()).reshape(Nt, Nm)))


def check_shift(F, rng, Nt=10, Nd=3, Nm=4):
    """Time-shift commutation F(S m) = S(F m), S delaying by one block (causal Toeplitz)."""
    blocks = rng.standard_normal((Nt, Nd, Nm))
    m = rng.standard_normal((Nt, Nm))
    Sm = np.zeros_like(m)
    Sm[1:] = m[:-1]
    Fm = F(blocks, m)
    SFm = np.zeros_like(Fm)
    SFm[1:] = Fm[:-1]
    return rel(F(blocks, Sm), SFm)


def check_linearity(F, rng, Nt=8, Nd=3, Nm=5, a=1.7, b=-0.6):
    blocks = rng.standard_normal((Nt, Nd, Nm))
    m1 = rng.standard_normal((Nt, Nm))
    m2 = rng.standard_normal((Nt, Nm))
    return rel(F(blocks, a * m1 + b * m2), a * F(blocks, m1) + b * F(blocks, m2))


TINY_SHAPES = [(1, 1, 1), (2, 1, 3), (3, 2, 2), (5, 7, 3), (8, 3, 7), (4, 7, 1), (1, 3, 5), (6, 2, 7)]


def run_all(F, FT, H, seed=0):
    """All checks; returns {name: worst error}."""
    rng = np.random.default_rng(seed)
    return {
        "bruteforce": check_bruteforce(F, FT, rng, TINY_SHAPES),
        "lti": check_lti(F, FT, rng),
        "scalar_convolution": check_scalar_convolution(F, FT, rng),
        "single_step": check_single_step(F, FT, rng),
        "delta": check_delta(F, FT, rng),
        "closed_form": check_closed_form(F, FT, rng),
        "adjoint": check_adjoint(F, FT, rng),
        "hessian": check_hessian(H, rng),
        "shift": check_shift(F, rng),
        "linearity": check_linearity(F, rng),
    }
