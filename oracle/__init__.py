"""FP64 CPU oracle for the block lower-triangular Toeplitz parameter-to-observable map.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the HIP product path
never does.  It shares no code with the HIP path (only the seeded input
generator in ``synth`` serves both).

What is computed is the plain definition, in FP64, with no FFT:

* The map F (paper section 2.1, eq. ShiftInvariance, with F_ij = B A^(i-j) C):
  a block lower-triangular Toeplitz matrix of Nt x Nt blocks, each Nd x Nm,
  given by its first block column F_0 .. F_{Nt-1}.  With 0-based time
  indices (output block i is the paper's d_{i+1}, input block j is m_j),
      (F m)_i = sum_{j=0}^{i} F_{i-j} m_j ,   i = 0 .. Nt-1.
* The adjoint F* (section 2.2 footnote, section 3.4): F is real, so F* = F^T,
  which is block upper-triangular Toeplitz:
      (F^T d)_j = sum_{i=j}^{Nt-1} F_{i-j}^T d_i .
* The Hessian (section 2.2, eq. LinearInverseProblem, with the noise and
  prior weights taken as scalars):  H m = F^T (noise_prec * F m) + prior_prec * m.
* Conjugate gradients on H x = b (section 2.2): textbook Hestenes-Stiefel CG
  in FP64 on the oracle's own H.

Layout: vectors are time-outer-space-inner (TOSI): m has shape [Nt][Nm]
(or [k][Nt][Nm] for k right-hand sides), d has shape [Nt][Nd]; blocks has
shape [Nt][Nd][Nm] with blocks[k] = F_k.

The block products use numpy's matmul as a library primitive; the sums are
taken lag by lag ("lag-outer": for each lag q, every output block i = j + q
receives F_q m_j), which is the definition's sum reordered only over its
terms.
"""
import numpy as np

__all__ = ["apply_F", "apply_FT", "apply_H", "dense_F", "entries_F", "entries_FT",
           "cg_solve", "rel_l2"]


def _as3(v):
    v = np.asarray(v, dtype=np.float64)
    return (v[None], True) if v.ndim == 2 else (v, False)


def apply_F(blocks, m):
    """(F m)_i = sum_{j<=i} F_{i-j} m_j  (eq. ShiftInvariance).  m: [..k][Nt][Nm] -> d: [..k][Nt][Nd]."""
    blocks = np.asarray(blocks, dtype=np.float64)
    Nt, Nd, Nm = blocks.shape
    m3, squeeze = _as3(m)
    assert m3.shape[1:] == (Nt, Nm), (m3.shape, blocks.shape)
    d = np.zeros((m3.shape[0], Nt, Nd))
    for q in range(Nt):                      # lag q = i - j
        # every d_i with i >= q receives F_q m_{i-q}
        d[:, q:, :] += m3[:, :Nt - q, :] @ blocks[q].T
    return d[0] if squeeze else d


def apply_FT(blocks, d):
    """(F^T d)_j = sum_{i>=j} F_{i-j}^T d_i  (block upper-triangular adjoint).  d: [..k][Nt][Nd] -> [..k][Nt][Nm]."""
    blocks = np.asarray(blocks, dtype=np.float64)
    Nt, Nd, Nm = blocks.shape
    d3, squeeze = _as3(d)
    assert d3.shape[1:] == (Nt, Nd), (d3.shape, blocks.shape)
    m = np.zeros((d3.shape[0], Nt, Nm))
    for q in range(Nt):                      # lag q = i - j
        m[:, :Nt - q, :] += d3[:, q:, :] @ blocks[q]
    return m[0] if squeeze else m


def apply_H(blocks, m, noise_prec=1.0, prior_prec=1.0):
    """H m = F^T (noise_prec F m) + prior_prec m  (eq. LinearInverseProblem, R = I)."""
    m = np.asarray(m, dtype=np.float64)
    return apply_FT(blocks, noise_prec * apply_F(blocks, m)) + prior_prec * m


def dense_F(blocks):
    """Brute force: assemble the full (Nd*Nt) x (Nm*Nt) matrix block by block.

    Block row i, block column j holds F_{i-j} when i >= j and zero otherwise.
    Pure Python loops over blocks; meant for tiny shapes only.
    """
    blocks = np.asarray(blocks, dtype=np.float64)
    Nt, Nd, Nm = blocks.shape
    A = np.zeros((Nt * Nd, Nt * Nm))
    for i in range(Nt):
        for j in range(Nt):
            if i >= j:
                A[i * Nd:(i + 1) * Nd, j * Nm:(j + 1) * Nm] = blocks[i - j]
    return A


def entries_F(blocks, m, idx):
    """Selected entries of F m: idx is a list of (i, s); entry = sum_{j<=i} F_{i-j}[s, :] . m_j."""
    blocks = np.asarray(blocks, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    out = np.empty(len(idx))
    for n, (i, s) in enumerate(idx):
        acc = 0.0
        for j in range(i + 1):
            acc += float(blocks[i - j, s, :] @ m[j])
        out[n] = acc
    return out


def entries_FT(blocks, d, idx):
    """Selected entries of F^T d: idx is a list of (j, p); entry = sum_{i>=j} F_{i-j}[:, p] . d_i."""
    blocks = np.asarray(blocks, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    Nt = blocks.shape[0]
    out = np.empty(len(idx))
    for n, (j, p) in enumerate(idx):
        acc = 0.0
        for i in range(j, Nt):
            acc += float(blocks[i - j, :, p] @ d[i])
        out[n] = acc
    return out


def cg_solve(apply_A, b, rtol=1e-8, max_iter=1000, x0=None):
    """Textbook conjugate gradients (Hestenes-Stiefel) in FP64 for an SPD operator.

    Stops when ||b - A x|| <= rtol ||b|| on the recurrence residual; returns
    (x, iterations, final true relative residual).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_A(x)
    p = r.copy()
    rr = float(np.vdot(r, r))
    bnorm = float(np.sqrt(np.vdot(b, b)))
    it = 0
    while it < max_iter and np.sqrt(rr) > rtol * bnorm:
        Ap = apply_A(p)
        alpha = rr / float(np.vdot(p, Ap))
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(np.vdot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    res = float(np.linalg.norm(b - apply_A(x)) / bnorm)
    return x, it, res


def rel_l2(y, y_ref):
    """||y - y_ref||_2 / ||y_ref||_2 over all entries, in FP64."""
    y = np.asarray(y, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    den = np.linalg.norm(y_ref.ravel())
    return float(np.linalg.norm((y - y_ref).ravel()) / (den if den > 0 else 1.0))
