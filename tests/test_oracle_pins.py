"""The FP64 oracle against what the paper and mathematics fix (CPU only).

Also plants plausible mistakes in copies of the oracle and checks that the
pins catch each of them, so that a passing oracle means something.
"""
import json
import os

import numpy as np
import pytest

import oracle
from tests import pins

TOL = 1e-12
HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_passes_every_pin():
    errs = pins.run_all(oracle.apply_F, oracle.apply_FT, oracle.apply_H)
    bad = {k: v for k, v in errs.items() if not v <= TOL}
    assert not bad, bad


def _mutant_lag_off_by_one(blocks, m):
    # uses F_{i-j+1}: the diagonal block dropped
    Nt = blocks.shape[0]
    d = np.zeros((Nt, blocks.shape[1]))
    for q in range(Nt - 1):
        d[q:, :] += m[:Nt - q, :] @ blocks[q + 1].T
    return d


def _mutant_upper(blocks, m):
    # anti-causal: (F m)_i = sum_{j>=i} F_{j-i} m_j
    Nt = blocks.shape[0]
    d = np.zeros((Nt, blocks.shape[1]))
    for q in range(Nt):
        d[:Nt - q, :] += m[q:, :] @ blocks[q].T
    return d


def _mutant_ft_as_f_transpose_time(blocks, d):
    # transposes each block but keeps the lower-triangular time structure
    Nt = blocks.shape[0]
    out = np.zeros((Nt, blocks.shape[2]))
    for q in range(Nt):
        out[q:, :] += d[:Nt - q, :] @ blocks[q]
    return out


def _mutant_ft_conj_sign(blocks, d):
    return -oracle.apply_FT(blocks, d)


def _mutant_h_no_prior(blocks, m, noise_prec=1.0, prior_prec=1.0):
    return oracle.apply_FT(blocks, noise_prec * oracle.apply_F(blocks, m))


def _mutant_h_prior_inside(blocks, m, noise_prec=1.0, prior_prec=1.0):
    return noise_prec * oracle.apply_FT(blocks, oracle.apply_F(blocks, m)) + prior_prec * noise_prec * m


def _mutant_truncated(blocks, m):
    # drops the last lag
    Nt = blocks.shape[0]
    d = np.zeros((Nt, blocks.shape[1]))
    for q in range(Nt - 1):
        d[q:, :] += m[:Nt - q, :] @ blocks[q].T
    return d


@pytest.mark.parametrize("F,FT,H", [
    (_mutant_lag_off_by_one, oracle.apply_FT, oracle.apply_H),
    (_mutant_upper, oracle.apply_FT, oracle.apply_H),
    (_mutant_truncated, oracle.apply_FT, oracle.apply_H),
    (oracle.apply_F, _mutant_ft_as_f_transpose_time, oracle.apply_H),
    (oracle.apply_F, _mutant_ft_conj_sign, oracle.apply_H),
    (oracle.apply_F, oracle.apply_FT, _mutant_h_no_prior),
    (oracle.apply_F, oracle.apply_FT, _mutant_h_prior_inside),
])
def test_pins_catch_planted_mistakes(F, FT, H):
    errs = pins.run_all(F, FT, H)
    assert max(errs.values()) > 1e-6, errs


def _fft_method(blocks, m, adjoint=False):
    """The paper's FFT method (section 2.4 and section 3.3-3.4) written with numpy.fft:
    zero-pad each time series to L = 2 Nt, transform, multiply per frequency by the
    transformed block column (conjugate transpose for the adjoint), inverse transform,
    keep the first Nt samples."""
    Nt = blocks.shape[0]
    L = 2 * Nt
    Fh = np.fft.rfft(blocks, n=L, axis=0)          # [Nt+1][Nd][Nm]
    xh = np.fft.rfft(m, n=L, axis=0)               # [Nt+1][n]
    if adjoint:
        yh = np.einsum("fsp,fs->fp", Fh.conj(), xh)
    else:
        yh = np.einsum("fsp,fp->fs", Fh, xh)
    return np.fft.irfft(yh, n=L, axis=0)[:Nt]


def test_fft_method_reading_matches_oracle():
    """Readings of the padding length (2 Nt, zeros appended), the real-to-complex
    Nt+1 bins, the 1/L normalisation on the inverse and the conjugate transpose
    for F^T reproduce the oracle exactly (to rounding)."""
    rng = np.random.default_rng(3)
    for (Nt, Nd, Nm) in [(1, 2, 3), (7, 3, 5), (32, 16, 64), (21, 4, 9)]:
        blocks = rng.standard_normal((Nt, Nd, Nm))
        m = rng.standard_normal((Nt, Nm))
        d = rng.standard_normal((Nt, Nd))
        assert pins.rel(_fft_method(blocks, m), oracle.apply_F(blocks, m)) < 1e-13
        assert pins.rel(_fft_method(blocks, d, adjoint=True), oracle.apply_FT(blocks, d)) < 1e-13


def test_scalar_toeplitz_circulant_embedding():
    """Section 2.4: a Toeplitz matrix embedded in a 2n circulant, diagonalised by the DFT;
    the matvec is the first block of IFFT(FFT(c) * FFT([x; 0]))."""
    rng = np.random.default_rng(4)
    n = 11
    col = rng.standard_normal(n)          # m_0 .. m_{n-1} (first column)
    row = np.concatenate([[col[0]], rng.standard_normal(n - 1)])  # m_0, m_{-1}, ...
    T = np.array([[col[i - j] if i >= j else row[j - i] for j in range(n)] for i in range(n)])
    c = np.concatenate([col, [0.0], row[1:][::-1]])        # first column of the circulant
    x = rng.standard_normal(n)
    u = np.concatenate([x, np.zeros(n)])
    y = np.fft.ifft(np.fft.fft(c) * np.fft.fft(u))[:n].real
    assert pins.rel(y, T @ x) < 1e-13
    # the lower-triangular case is the oracle with Nd = Nm = 1
    assert pins.rel(oracle.apply_F(col.reshape(n, 1, 1), x.reshape(n, 1)).ravel(),
                    np.tril(T) @ x) < 1e-13


def test_multi_rhs_is_columnwise():
    rng = np.random.default_rng(5)
    blocks = rng.standard_normal((6, 3, 4))
    M = rng.standard_normal((3, 6, 4))
    D = rng.standard_normal((3, 6, 3))
    FM = oracle.apply_F(blocks, M)
    FTD = oracle.apply_FT(blocks, D)
    for r in range(3):
        assert pins.rel(FM[r], oracle.apply_F(blocks, M[r])) == 0.0
        assert pins.rel(FTD[r], oracle.apply_FT(blocks, D[r])) == 0.0


def test_sampled_entries_match_full():
    rng = np.random.default_rng(6)
    Nt, Nd, Nm = 9, 4, 7
    blocks = rng.standard_normal((Nt, Nd, Nm))
    m = rng.standard_normal((Nt, Nm))
    d = rng.standard_normal((Nt, Nd))
    Fm = oracle.apply_F(blocks, m)
    FTd = oracle.apply_FT(blocks, d)
    idx = [(i, s) for i in range(Nt) for s in range(Nd)]
    assert pins.rel(oracle.entries_F(blocks, m, idx), Fm.ravel()) < 1e-14
    idx = [(j, p) for j in range(Nt) for p in range(Nm)]
    assert pins.rel(oracle.entries_FT(blocks, d, idx), FTd.ravel()) < 1e-14


def test_cg_matches_dense_solve():
    rng = np.random.default_rng(7)
    Nt, Nd, Nm = 6, 2, 5
    blocks = rng.standard_normal((Nt, Nd, Nm))
    b = rng.standard_normal((Nt, Nm))
    noise_prec, prior_prec = 4.0, 0.1
    A = pins.dense_matrix(blocks)
    Hd = noise_prec * A.T @ A + prior_prec * np.eye(A.shape[1])
    x_ref = np.linalg.solve(Hd, b.ravel()).reshape(Nt, Nm)
    x, it, res = oracle.cg_solve(lambda v: oracle.apply_H(blocks, v, noise_prec, prior_prec), b,
                                 rtol=1e-13, max_iter=500)
    assert res < 1e-12
    assert pins.rel(x, x_ref) < 1e-9
    assert it <= 500


def test_golden_fp64_small():
    """Regression against stored values written by tests/golden/make_golden.py (oracle only)."""
    import synth
    with open(os.path.join(HERE, "golden", "fp64_small.json")) as f:
        g = json.load(f)
    w = synth.WORKLOADS["fp64-small"]
    blocks = synth.blocks(w["Nt"], w["Nd"], w["Nm"], w["tau"])
    m = synth.vectors(1, w["Nt"], w["Nm"], synth.STREAM_M)[0]
    d = synth.vectors(1, w["Nt"], w["Nd"], synth.STREAM_D)[0]
    Fm = oracle.apply_F(blocks, m).ravel()
    FTd = oracle.apply_FT(blocks, d).ravel()
    Hm = oracle.apply_H(blocks, m, w["noise_prec"], w["prior_prec"]).ravel()
    for name, v in (("Fm", Fm), ("FTd", FTd), ("Hm", Hm)):
        ent = g[name]
        idx = np.array(ent["index"])
        np.testing.assert_allclose(v[idx], np.array(ent["value"]), rtol=1e-13, atol=1e-13)
        assert abs(np.linalg.norm(v) - ent["norm"]) <= 1e-12 * ent["norm"]


# ---- the dense assembler ------------------------------------------------------------
# oracle.dense_F assembles the block matrix of eq. ShiftInvariance (section 2.1): block row i,
# block column j holds F_{i-j} for i >= j and zero above the block diagonal.  It is pinned to
# facts that do not go through the oracle's own code: scipy's Toeplitz constructor for
# Nd = Nm = 1, time stepping of an LTI system (section 2.1), the entry-by-entry assembly in
# tests/pins.py, and the delta property (block column 0 is the first block column).

def _dense_pins(dense):
    """Worst relative error of ``dense`` over every pin of the assembler."""
    import scipy.linalg
    rng = np.random.default_rng(11)
    worst = 0.0
    for Nt in (1, 2, 5, 9):
        f = rng.standard_normal(Nt)
        T = scipy.linalg.toeplitz(f, np.zeros(Nt))      # lower-triangular Toeplitz
        worst = max(worst, pins.rel(dense(f.reshape(Nt, 1, 1)), T))
    for (Nt, Nd, Nm) in pins.TINY_SHAPES:
        blocks = rng.standard_normal((Nt, Nd, Nm))
        A = dense(blocks)
        if A.shape != (Nt * Nd, Nt * Nm):
            return np.inf
        worst = max(worst, pins.rel(A, pins.dense_matrix(blocks)))
        # block column 0 is the first block column, stacked over block rows
        worst = max(worst, pins.rel(A[:, :Nm], blocks.reshape(Nt * Nd, Nm)))
    A_, B, C, blocks = pins.lti_system(rng, 7, 3, 4, 10)
    m = rng.standard_normal((10, 4))
    u = np.zeros(7)
    d = np.empty((10, 3))
    for k in range(10):
        u = A_ @ u + C @ m[k]
        d[k] = B @ u
    worst = max(worst, pins.rel(dense(blocks) @ m.ravel(), d.ravel()))
    return worst


def test_dense_assembler_pinned():
    assert _dense_pins(oracle.dense_F) < 1e-14


def _dense_mutant_upper(blocks):
    # the triangle mirrored: F_{j-i} placed where j >= i
    Nt, Nd, Nm = blocks.shape
    A = np.zeros((Nt * Nd, Nt * Nm))
    for i in range(Nt):
        for j in range(Nt):
            if i <= j:
                A[i * Nd:(i + 1) * Nd, j * Nm:(j + 1) * Nm] = blocks[j - i]
    return A


def _dense_mutant_strict(blocks):
    # diagonal blocks dropped (i > j instead of i >= j)
    Nt, Nd, Nm = blocks.shape
    A = np.zeros((Nt * Nd, Nt * Nm))
    for i in range(Nt):
        for j in range(i):
            A[i * Nd:(i + 1) * Nd, j * Nm:(j + 1) * Nm] = blocks[i - j]
    return A


def _dense_mutant_lag(blocks):
    # block (i, j) takes F_{i-j-1}: the block column shifted down one block
    Nt, Nd, Nm = blocks.shape
    A = np.zeros((Nt * Nd, Nt * Nm))
    for i in range(Nt):
        for j in range(i):
            A[i * Nd:(i + 1) * Nd, j * Nm:(j + 1) * Nm] = blocks[i - j - 1]
    return A


@pytest.mark.parametrize("dense", [_dense_mutant_upper, _dense_mutant_strict, _dense_mutant_lag])
def test_dense_assembler_pins_catch_planted_mistakes(dense):
    assert _dense_pins(dense) > 1e-6
