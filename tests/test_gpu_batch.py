"""Batched blocks (Section 3.2.2 independent-block form): one launch steps every
block; each block must match the FP64 oracle's step of that block alone.

Tolerances as for the single-grid parity tests: solved to a 1e-12 relative
residual in the Jacobi-scaled norm, the relative L2 error of E and T per block
is <= 1e-10 (FP64 and mixed precision); elementwise <= 1e-7."""
import numpy as np
import pytest

import fld_workloads as W
from oracle import fld_oracle as O
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PARITY = dict(rel_tol=1e-12, norm=1)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _blocks(shapes, first=0):
    return [W.make_c4_block(first + b, nx, ny) for b, (nx, ny) in enumerate(shapes)]


def _packed(blocks):
    f = {k: _dev(np.concatenate([getattr(b, k).ravel() for b in blocks]))
         for k in ("E", "T", "rho", "kappa_R", "kappa_P", "c_v")}
    f["ghost_E"] = _dev(np.concatenate([b.ghost_E for b in blocks]))
    return f


def _make_batch(fld, blocks, threads=None, **opt):
    nx = [b.nx for b in blocks]
    ny = [b.ny for b in blocks]
    dx = [b.x_faces[1] - b.x_faces[0] for b in blocks]
    dy = [b.y_faces[1] - b.y_faces[0] for b in blocks]
    bt = fld.Batch(nx, ny, dx, dy, None, fld.default_options(**opt))
    if threads:
        bt.threads = threads
    return bt


def _run(fld, blocks, threads=None, nsteps=1, multi=False, **opt):
    bt = _make_batch(fld, blocks, threads, **opt)
    f = _packed(blocks)
    args = (f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], blocks[0].dt, f["ghost_E"])
    if multi:
        infos = bt.steps(nsteps, f["E"], f["T"], *args, check=False)
    else:
        for _ in range(nsteps):
            infos = bt.step(f["E"], f["T"], *args, check=False)
    torch.cuda.synchronize()
    E, T = f["E"].cpu().numpy(), f["T"].cpu().numpy()
    bt.close()
    return E, T, infos


def _split(a, blocks):
    out, o = [], 0
    for b in blocks:
        n = b.nx * b.ny
        out.append(a[o:o + n].reshape(b.ny, b.nx))
        o += n
    return out


SHAPES = [(16, 16), (128, 32), (48, 96), (1, 1), (1, 37), (29, 1), (3, 5), (65, 17), (96, 128), (8, 8),
          (9, 7), (128, 128)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_matches_oracle_per_block(lib, prec):
    blocks = _blocks(SHAPES)
    E, T, infos = _run(lib, blocks, precision=prec, **PARITY)
    assert [i["status"] for i in infos] == [0] * len(blocks), infos
    for b, Eb, Tb, inf in zip(blocks, _split(E, blocks), _split(T, blocks), infos):
        r = O.step_problem(b)
        assert rel_l2(Eb, r.E) < 1e-10, (b.name, b.nx, b.ny, inf)
        assert rel_l2(Tb, r.T) < 1e-10, (b.name, b.nx, b.ny)
        assert np.max(np.abs(Eb - r.E) / np.abs(r.E)) < 1e-7


@pytest.mark.parametrize("threads", [256, 1024])
def test_batch_workgroup_sizes_agree(lib, threads):
    blocks = _blocks(SHAPES[:6])
    E0, T0, _ = _run(lib, blocks, threads=512, precision="mixed", **PARITY)
    E1, T1, infos = _run(lib, blocks, threads=threads, precision="mixed", **PARITY)
    assert all(i["status"] == 0 for i in infos)
    assert rel_l2(E1, E0) < 1e-11 and rel_l2(T1, T0) < 1e-11


def test_batch_deterministic_and_graph_steps_match(lib):
    blocks = _blocks(SHAPES[:5], first=20)
    E1, T1, _ = _run(lib, blocks, nsteps=3, precision="mixed", **PARITY)
    E2, T2, _ = _run(lib, blocks, nsteps=3, precision="mixed", **PARITY)
    E3, T3, i3 = _run(lib, blocks, nsteps=3, multi=True, precision="mixed", **PARITY)
    assert np.array_equal(E1, E2) and np.array_equal(T1, T2)
    assert np.array_equal(E1, E3) and np.array_equal(T1, T3)
    assert all(i["status"] == 0 for i in i3)


def test_batch_multistep_vs_oracle(lib):
    blocks = _blocks([(32, 48), (16, 16), (64, 32)], first=40)
    E, T, _ = _run(lib, blocks, nsteps=5, multi=True, precision="mixed", **PARITY)
    for b, Eb, Tb in zip(blocks, _split(E, blocks), _split(T, blocks)):
        Eo, To = b.E, b.T
        for _ in range(5):
            r = O.step_problem(b, Eo, To)
            Eo, To = r.E, r.T
        assert rel_l2(Eb, Eo) < 1e-9 and rel_l2(Tb, To) < 1e-9


@pytest.mark.parametrize("shape", [(100, 60), (60, 100), (40, 24)])
def test_batch_single_ragged_block_fp64(lib, shape):
    """One block alone, so it sits at offset 0 of every array, with line counts
    that leave idle lanes in the last pass of its line sweeps (binary64 takes
    the branch-free loads): regression for a load before the arrays' start."""
    blocks = _blocks([shape], first=70)
    print(f"[batch] fp64 single block {shape}", flush=True)
    E, T, infos = _run(lib, blocks, precision="fp64", **PARITY)
    assert infos[0]["status"] == 0, infos
    r = O.step_problem(blocks[0])
    assert rel_l2(E.reshape(shape[1], shape[0]), r.E) < 1e-10
    assert rel_l2(T.reshape(shape[1], shape[0]), r.T) < 1e-10


def test_batch_matches_single_grid_solver(lib):
    """The same block through fld_step (one context) and through the batch."""
    from gpu_helpers import gpu_step
    b = W.make_c4_block(3, 64, 48)
    E, T, _ = _run(lib, [b], precision="mixed", **PARITY)
    Es, Ts, info = gpu_step(lib, torch, b, precision="mixed", **PARITY)
    assert info["status"] == 0
    assert rel_l2(E.reshape(b.ny, b.nx), Es) < 1e-11


def test_batch_bad_block_is_isolated(lib):
    blocks = _blocks([(16, 16), (32, 16), (16, 32)], first=60)
    f = _packed(blocks)
    f["rho"][16 * 16 + 5] = float("nan")  # a cell of block 1
    bt = _make_batch(lib, blocks, precision="mixed", **PARITY)
    infos = bt.step(f["E"], f["T"], f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], blocks[0].dt, f["ghost_E"],
                    check=False)
    assert [i["status"] for i in infos] == [0, 6, 0]
    E = f["E"].cpu().numpy()
    r = O.step_problem(blocks[2])
    assert rel_l2(_split(E, blocks)[2], r.E) < 1e-10
    bt.close()


def test_batch_invalid_arguments(lib):
    with pytest.raises(lib.FLDError):
        lib.Batch([0], [4], [1.0], [1.0])
    with pytest.raises(lib.FLDError):
        lib.Batch([513], [4], [1.0], [1.0])
    with pytest.raises(lib.FLDError):
        lib.Batch([4], [4], [-1.0], [1.0])
    with pytest.raises(lib.FLDError):
        lib.Batch([4], [4], [1.0], [1.0], options=lib.default_options(smoother=1))
    blocks = _blocks([(8, 8)])
    bt = _make_batch(lib, blocks)
    f = _packed(blocks)
    with pytest.raises(lib.FLDError):
        bt.step(f["E"], f["T"], f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], 1e4, None)
    with pytest.raises(lib.FLDError):
        bt.step(f["E"], f["T"], f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], -1.0, f["ghost_E"])
    with pytest.raises(lib.FLDError):
        bt.threads = 300
    bt.close()


def test_batch_full_c4_sampled(lib):
    """All 256 blocks of the c4 recipe in one launch, in the configuration the
    benchmark times (mixed, 1e-10 in the per-volume norm): every block
    converges; eight sampled blocks re-solved at the parity tolerance match
    the oracle."""
    batch = W.make_c4()
    blocks = batch.blocks
    E, T, infos = _run(lib, blocks, precision="mixed", rel_tol=1e-10, norm=0)
    assert all(i["status"] == 0 for i in infos)
    assert max(i["rel_resid"] for i in infos) <= 1e-10
    E, T, infos = _run(lib, blocks, precision="mixed", **PARITY)
    assert all(i["status"] == 0 for i in infos)
    rng = np.random.default_rng(7)
    Es, Ts = _split(E, blocks), _split(T, blocks)
    for k in rng.choice(len(blocks), size=8, replace=False):
        r = O.step_problem(blocks[k])
        assert rel_l2(Es[k], r.E) < 1e-10, (k, blocks[k].nx, blocks[k].ny)
        assert rel_l2(Ts[k], r.T) < 1e-10
