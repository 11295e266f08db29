"""Setup in rectangles, from the last block row, and persistence of the transformed operator
(needs an MI355X).

Every (sensor, parameter) series is transformed on its own, so an operator filled rectangle
by rectangle must store the very bytes of the one-shot setup; so must one set up from the
last block row (section 2.3: Nd adjoint solves give that row, Nm forward solves the first
block column); and a saved and reloaded operator must hold them again.  The stored bytes
are compared through btoep_save files.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import make, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 3e-3}
STORAGES = ["f64", "f32", "bf16"]
# a single-pass shape with ragged rectangles and row padding (Nm = 301 -> rows of 304), and
# a series long enough for the four-step transforms (Nt = 5000)
SHAPES = [(37, 5, 301), (5000, 3, 70)]


def stored(bt, op, path):
    bt.btoep_save(op, str(path))
    return path.read_bytes()


def cuts(n, inner):
    return [0] + [c for c in inner if 0 < c < n] + [n]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("where", ["host", "device"])
def test_rectangles_store_the_one_shot_bytes(bt, tmp_path, shape, storage, where):
    Nt, Nd, Nm = shape
    print("rectangles", shape, storage, where, flush=True)
    blocks = synth.blocks(Nt, Nd, Nm, tau=Nt / 6, seed=91)
    want = stored(bt, make(bt, blocks, storage), tmp_path / "ref.bin")
    src = blocks if where == "host" else torch.from_numpy(blocks).cuda()
    sc, pc = cuts(Nd, [2]), cuts(Nm, [64, 173])
    rects = [(a, b, c, d) for a, b in zip(sc, sc[1:]) for c, d in zip(pc, pc[1:])]
    order = np.random.default_rng(5).permutation(len(rects))
    op = bt.btoep_create_empty(Nt, Nd, Nm, storage)
    for n, i in enumerate(order):
        s0, s1, p0, p1 = rects[i]
        sub = src[:, s0:s1, p0:p1]  # a strided view of the whole block column
        if n % 2:
            sub = np.ascontiguousarray(sub) if where == "host" else sub.contiguous()
        bt.btoep_set_blocks(op, s0, p0, sub)
    assert stored(bt, op, tmp_path / "op.bin") == want


@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("where", ["host", "device"])
def test_last_block_row_from_the_assembled_matrix(bt, tmp_path, storage, where):
    """The last block row is cut out of the oracle's assembled matrix and handed over as is."""
    Nt, Nd, Nm = 23, 4, 130
    blocks = synth.blocks(Nt, Nd, Nm, tau=5.0, seed=92)
    A = oracle.dense_F(blocks)
    row = A[(Nt - 1) * Nd:, :].reshape(Nd, Nt, Nm).transpose(1, 0, 2)  # [j][s][p] = block (Nt-1, j)
    row = np.ascontiguousarray(row)
    want = stored(bt, make(bt, blocks, storage), tmp_path / "ref.bin")
    op = bt.btoep_create_empty(Nt, Nd, Nm, storage)
    bt.btoep_set_blocks(op, 0, 0, row if where == "host" else torch.from_numpy(row).cuda(), order="last_row")
    assert stored(bt, op, tmp_path / "op.bin") == want
    m = synth.vectors(1, Nt, Nm, stream=93)[0]
    got = bt.btoep_apply_F(op, to_dev(m, op.vector_dtype))
    assert oracle.rel_l2(got.double().cpu().numpy().reshape(-1), A @ m.reshape(-1)) <= TOL[storage]


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_last_block_row_of_a_long_series(bt, tmp_path, storage):
    """Four-step setup reading its input backwards, in two sensor rectangles."""
    Nt, Nd, Nm = 5000, 3, 70
    blocks = synth.blocks(Nt, Nd, Nm, tau=Nt / 6, seed=94)
    want = stored(bt, make(bt, blocks, storage), tmp_path / "ref.bin")
    row = np.ascontiguousarray(blocks[::-1])
    op = bt.btoep_create_empty(Nt, Nd, Nm, storage)
    bt.btoep_set_blocks(op, 0, 0, row[:, :1], order="last_row")
    bt.btoep_set_blocks(op, 1, 0, torch.from_numpy(row).cuda()[:, 1:], order="last_row")
    assert stored(bt, op, tmp_path / "op.bin") == want


@pytest.mark.parametrize("storage", STORAGES)
def test_unset_rectangles_are_zero_blocks(bt, storage):
    Nt, Nd, Nm = 37, 5, 301
    blocks = synth.blocks(Nt, Nd, Nm, tau=Nt / 6, seed=95)
    op = bt.btoep_create_empty(Nt, Nd, Nm, storage)
    m = synth.vectors(1, Nt, Nm, stream=96)[0]
    d = synth.vectors(1, Nt, Nd, stream=97)[0]
    empty = bt.btoep_apply_F(op, to_dev(m, op.vector_dtype))
    assert torch.count_nonzero(empty).item() == 0
    part = np.zeros_like(blocks)
    for s0, s1, p0, p1 in [(0, 2, 64, 173), (2, 5, 0, 64), (4, 5, 250, 301)]:
        bt.btoep_set_blocks(op, s0, p0, blocks[:, s0:s1, p0:p1])
        part[:, s0:s1, p0:p1] = blocks[:, s0:s1, p0:p1]
    got_F = bt.btoep_apply_F(op, to_dev(m, op.vector_dtype)).double().cpu().numpy()
    got_FT = bt.btoep_apply_FT(op, to_dev(d, op.vector_dtype)).double().cpu().numpy()
    assert got_F.shape == (Nt, Nd) and got_FT.shape == (Nt, Nm)
    assert oracle.rel_l2(got_F, oracle.apply_F(part, m)) <= TOL[storage]
    assert oracle.rel_l2(got_FT, oracle.apply_FT(part, d)) <= TOL[storage]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("storage", STORAGES)
def test_save_and_load_give_the_same_operator(bt, tmp_path, shape, storage):
    Nt, Nd, Nm = shape
    print("persistence", shape, storage, flush=True)
    blocks = synth.blocks(Nt, Nd, Nm, tau=Nt / 6, seed=98)
    op = make(bt, blocks, storage)
    first = stored(bt, op, tmp_path / "a.bin")
    assert len(first) == 64 + op.info["nfreq"] * Nd * Nm * {"f64": 16, "f32": 8, "bf16": 4}[storage]
    op2 = bt.btoep_load(str(tmp_path / "a.bin"))
    assert op2.info == op.info
    assert stored(bt, op2, tmp_path / "b.bin") == first
    vt = op.vector_dtype
    m = to_dev(synth.vectors(2, Nt, Nm, stream=99), vt)
    d = to_dev(synth.vectors(2, Nt, Nd, stream=100), vt)
    assert torch.equal(bt.btoep_apply_F(op, m), bt.btoep_apply_F(op2, m))
    assert torch.equal(bt.btoep_apply_FT(op, d), bt.btoep_apply_FT(op2, d))
    assert torch.equal(bt.btoep_apply_H(op, m, 2.0, 0.5), bt.btoep_apply_H(op2, m, 2.0, 0.5))
    got = bt.btoep_apply_F(op2, m).double().cpu().numpy()
    assert oracle.rel_l2(got, oracle.apply_F(blocks, m.double().cpu().numpy())) <= TOL[storage]


def test_set_blocks_rejects_bad_rectangles(bt):
    import ctypes
    lib = bt.load_library()
    op = bt.btoep_create_empty(8, 3, 20, "f32")
    buf = torch.zeros((8, 3, 20), dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())

    def call(s0, ns, p0, np_, ld_t, ld_s, order=0):
        return lib.btoep_set_blocks(op.handle, s0, ns, p0, np_, p, ld_t, ld_s, order, 1, None)

    assert call(0, 3, 0, 20, 60, 20) == 0
    assert call(1, 3, 0, 20, 60, 20) == 1  # past the last sensor
    assert call(0, 3, 5, 16, 60, 20) == 1  # past the last parameter
    assert call(0, 0, 0, 20, 60, 20) == 1
    assert call(0, 3, 0, 20, 60, 19) == 1  # sensor rows overlap
    assert call(0, 3, 0, 20, 59, 20) == 1  # time rows overlap
    assert call(0, 3, 0, 20, 60, 20, order=2) == 1
    with pytest.raises(ValueError):
        bt.btoep_set_blocks(op, 0, 0, np.zeros((7, 3, 20)))
