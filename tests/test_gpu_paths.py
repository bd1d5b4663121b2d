"""The kernel paths the large workloads take, against the oracle.

* Rows of 4096 cells (the 4096 x 2048 stress recipe's r-lines: whole-chunk
  line solves with cyclic reduction of 512 chunk interfaces in LDS) and of
  2048 cells (the 2048 x 512 recipe's r-lines and the stress recipe's
  theta-lines), in both precisions, and the band-fused against the split
  sweeps after a fixed number of iterations at 4096 cells.
* The 2048 x 512 spherical recipe at full size, one step, against the
  oracle's direct solve.
* Theta slabs of the 4096 x 2048 stress recipe at full resolution (the share
  of one GPU in a slab decomposition), both about the equator: 4096 x 256 for
  one step (two sequential V-cycles, the benchmark's cycle), and 4096 x 128
  for ten graph-replayed steps (K-cycle) against ten oracle steps.
* The full 4096 x 2048 stress recipe, one step in the benchmark's schedule:
  the assembled operator elementwise against the oracle's assembly, the GPU
  solution's residual in the oracle's own system, and T^{n+1} against the
  oracle's gas update of the GPU's E (the oracle cannot solve this size
  directly: these properties hold at any size).
* Every one of the 256 blocks of the batched recipe against its own oracle
  step.

Tolerances: relative L2 error of E and T <= 1e-10 where binary64 allows it.
The stress recipe's full-resolution rows (optically thin shells whose face
conductances exceed the cell masses by up to 1e11) put the binary64 floor of
the Jacobi-scaled residual near 3e-11 even for the oracle's refined solution:
there the GPU stops at 3e-11 (the 256-row slab; errors ~5e-11), at 2e-10
(the 128-row slab, whose floor lies near 1e-10: ten compounded steps, bound
1e-9) or at the benchmark's 1e-10 (the 4096 x 64 strip, whose two polar rows
of 1/64 of pi are the worst conditioned: two solutions at that floor, the
GPU's and the oracle's, differ by ~4e-10, so its bound is 1e-9)."""
import numpy as np
import pytest

import fld_workloads as W
from oracle import fld_oracle as O
from gpu_helpers import gpu_step, make_ctx, rel_l2, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PARITY = dict(rel_tol=1e-12, norm=1)
# the stress recipe at full radial resolution: just above the binary64 floor
PARITY_C5 = dict(rel_tol=3e-11, norm=1)


@pytest.mark.parametrize("name,kw,opt,bound", [
    ("c5", dict(nx=4096, ny=64), dict(rel_tol=1e-10, norm=1), 1e-9),
    ("c3", dict(nx=2048, ny=128), PARITY, 1e-10),
    ("c5", dict(nx=64, ny=2048), PARITY, 1e-10)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_long_rows_match_oracle(lib, name, kw, opt, bound, prec):
    prob = W.make(name, **kw)
    print(f"[long rows] {name} {prob.nx}x{prob.ny} {prec}", flush=True)
    ref = O.step_problem(prob)
    E, T, info = gpu_step(lib, torch, prob, precision=prec, **opt)
    print(info["inner_iters"], info["rel_resid"], rel_l2(E, ref.E), rel_l2(T, ref.T), flush=True)
    assert info["status"] == 0
    assert rel_l2(E, ref.E) < bound and rel_l2(T, ref.T) < bound


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_band_fused_against_split_at_4096(lib, prec):
    prob = W.make_c5(nx=4096, ny=64)
    print(f"[fused vs split] 4096x64 {prec}", flush=True)
    opt = dict(precision=prec, max_inner=3, norm=1)
    E1, _, i1 = gpu_step(lib, torch, prob, smoother=0, **opt)
    E2, _, i2 = gpu_step(lib, torch, prob, smoother=2, **opt)
    assert i1["inner_iters"] == i2["inner_iters"] == 3
    E0 = np.asarray(prob.E)
    assert rel_l2(E1 - E0, E2 - E0) < (1e-10 if prec == "fp64" else 1e-4)


@pytest.fixture(scope="module")
def c3_full():
    prob = W.make_c3()
    print("[c3 full] oracle", flush=True)
    return prob, O.step_problem(prob)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_c3_full_size_one_step(lib, c3_full, prec):
    prob, ref = c3_full
    print(f"[c3 full] 2048x512 {prec}", flush=True)
    E, T, info = gpu_step(lib, torch, prob, precision=prec, **PARITY)
    print(info["inner_iters"], rel_l2(E, ref.E), rel_l2(T, ref.T), flush=True)
    assert info["status"] == 0
    assert rel_l2(E, ref.E) < 1e-10 and rel_l2(T, ref.T) < 1e-10


@pytest.fixture(scope="module")
def c5_full():
    return W.make_c5()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_c5_slab_one_step(lib, c5_full, prec):
    prob = W.theta_slab(c5_full, 896, 1152)
    print(f"[c5 slab] {prob.nx}x{prob.ny} {prec}", flush=True)
    ref = O.step_problem(prob)
    E, T, info = gpu_step(lib, torch, prob, precision=prec, mg_cycle=2, **PARITY_C5)
    print(info["inner_iters"], info["rel_resid"], rel_l2(E, ref.E), rel_l2(T, ref.T), flush=True)
    assert info["status"] == 0
    assert rel_l2(E, ref.E) < 1e-10 and rel_l2(T, ref.T) < 1e-10


@pytest.fixture(scope="module")
def c5_slab_ten_steps(c5_full):
    prob = W.theta_slab(c5_full, 960, 1088)
    print(f"[c5 slab x10] oracle {prob.nx}x{prob.ny}", flush=True)
    E, T = prob.E, prob.T
    for _ in range(10):
        r = O.step_problem(prob, E=E, T=T)
        E, T = r.E, r.T
    return prob, E, T


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_c5_slab_ten_graph_steps(lib, c5_slab_ten_steps, prec):
    prob, Eref, Tref = c5_slab_ten_steps
    print(f"[c5 slab x10] {prec}", flush=True)
    ctx = make_ctx(lib, prob, precision=prec, mg_cycle=1, rel_tol=2e-10, norm=1)
    t = to_dev(prob, torch)
    infos = ctx.steps(10, t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, t["ghost_E"],
                      check=False)
    torch.cuda.synchronize()
    E, T = t["E"].cpu().numpy(), t["T"].cpu().numpy()
    ctx.close()
    print([(i["status"], i["inner_iters"], i["rel_resid"]) for i in infos], rel_l2(E, Eref), rel_l2(T, Tref),
          flush=True)
    assert all(i["status"] == 0 for i in infos)
    assert rel_l2(E, Eref) < 1e-9 and rel_l2(T, Tref) < 1e-9  # ten steps at the binary64 floor


def test_c5_full_size_properties(lib, c5_full):
    """One step of the full stress grid in the benchmark's schedule (mixed,
    two sequential V-cycles, scaled norm 1e-10)."""
    prob = c5_full
    print("[c5 full] 4096x2048 mixed", flush=True)
    ctx = make_ctx(lib, prob, precision="mixed", mg_cycle=2, rel_tol=1e-10, norm=1)
    t = to_dev(prob, torch)
    ctx.assemble(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, t["ghost_E"])
    op = {k: v.cpu().numpy() for k, v in ctx.get_operator().items()}
    E = t["E"].clone()
    info = ctx.solve(E, check=False)
    Tn = t["T"].clone()
    ctx.gas_update(E, Tn)
    torch.cuda.synchronize()
    E, Tn = E.cpu().numpy(), Tn.cpu().numpy()
    ctx.close()
    del t
    assert info["status"] == 0 and info["rel_resid"] <= 1e-10
    A = O.assemble_problem(prob)
    ref_We = np.zeros_like(A.diag)
    ref_We[:, :-1] = A.W_x[:, 1:-1]
    ref_Wn = np.zeros_like(A.diag)
    ref_Wn[:-1, :] = A.W_y[1:-1, :]
    for got, want, nm in ((op["W_e"], ref_We, "W_e"), (op["W_n"], ref_Wn, "W_n"),
                          (op["diag"], A.diag, "diag"), (op["rhs"], A.rhs, "rhs")):
        err = np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300))
        assert err < 1e-12, (nm, err)
    res = O.residual_scaled(A, E)
    print("oracle residual of the GPU solution", res, "reported", info["rel_resid"], flush=True)
    # the oracle's binary64 evaluation of the residual has its own floor near
    # 1e-10 on this grid (the GPU's flux form rounds less)
    assert res <= 3e-10
    np.testing.assert_allclose(Tn, O.gas_update(A, prob.T, E), rtol=1e-13)


def _split(x, blocks):
    out, o = [], 0
    for b in blocks:
        n = b.nx * b.ny
        out.append(x[o:o + n].reshape(b.ny, b.nx))
        o += n
    return out


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_c4_every_block(lib, prec):
    batch = W.make_c4()
    blocks = batch.blocks
    print(f"[c4 all blocks] {len(blocks)} {prec}", flush=True)
    nx = [b.nx for b in blocks]
    ny = [b.ny for b in blocks]
    dx = [b.x_faces[1] - b.x_faces[0] for b in blocks]
    dy = [b.y_faces[1] - b.y_faces[0] for b in blocks]
    bt = lib.Batch(nx, ny, dx, dy, None, lib.default_options(precision=prec, **PARITY))
    dev = {k: torch.tensor(batch.packed(k), dtype=torch.float64, device="cuda")
           for k in ("E", "T", "rho", "kappa_R", "kappa_P", "c_v", "ghost_E")}
    infos = bt.step(dev["E"], dev["T"], dev["rho"], dev["kappa_R"], dev["kappa_P"], dev["c_v"], blocks[0].dt,
                    dev["ghost_E"], check=False)
    torch.cuda.synchronize()
    bt.close()
    assert all(i["status"] == 0 for i in infos)
    Es, Ts = _split(dev["E"].cpu().numpy(), blocks), _split(dev["T"].cpu().numpy(), blocks)
    worst = 0.0
    for k, b in enumerate(blocks):
        r = O.step_problem(b)
        e = max(rel_l2(Es[k], r.E), rel_l2(Ts[k], r.T))
        worst = max(worst, e)
        assert e < 1e-10, (k, b.nx, b.ny, e)
    print("worst block", worst, flush=True)
