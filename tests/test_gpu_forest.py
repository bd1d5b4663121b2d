"""The block forest solved as one matrix across levels (fld_forest_*,
Section 3.2.2) against the forest oracle: refined patches at levels 1 and 2,
every domain boundary kind, several steps, and the uniform limit against
the single-grid step.  Tolerance as the other parity tests: solves to a
1e-12 scaled residual, relative L2 error of E and T <= 1e-10."""
import numpy as np
import pytest

import fld_workloads as W
from oracle import fld_forest as FF
from oracle import fld_oracle as O
from gpu_helpers import make_ctx, rel_l2, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PAR = dict(precision="fp64", rel_tol=1e-12, norm=1, max_inner=20000)


def fields_for(n, seed, T0=5e3, rho0=1e-9):
    rng = np.random.default_rng(seed)
    rho = rho0 * np.exp(0.8 * rng.normal(size=n))
    T = T0 * np.exp(0.3 * rng.normal(size=n))
    kap = np.clip(1e22 * rho * T ** -3.5, 1e-4, 1e4)
    return dict(E=O.A_RAD * T ** 4 * np.exp(0.2 * rng.normal(size=n)), T=T, rho=rho, kappa_R=kap,
                kappa_P=kap.copy(), c_v=np.full(n, 1e8))


def nested_patches(nx0, ny0):
    """A level-1 patch over the middle half of the domain with a level-2 patch
    over its middle half, the rest at level 0, all blocks 2:1 balanced."""
    a, b = nx0 // 4, 3 * nx0 // 4
    c, d = ny0 // 4, 3 * ny0 // 4
    blocks = [(0, 0, 0, nx0, c), (0, 0, d, nx0, ny0 - d), (0, 0, c, a, d - c), (0, b, c, nx0 - b, d - c)]
    # level 1 covers coarse [a, b) x [c, d): fine [2a, 2b) x [2c, 2d); level 2 covers its middle half
    A, B, C, D = 2 * a, 2 * b, 2 * c, 2 * d
    qa, qb = A + (B - A) // 4, A + 3 * (B - A) // 4
    qc, qd = C + (D - C) // 4, C + 3 * (D - C) // 4
    blocks += [(1, A, C, B - A, qc - C), (1, A, qd, B - A, D - qd), (1, A, qc, qa - A, qd - qc),
               (1, qb, qc, B - qb, qd - qc), (2, 2 * qa, 2 * qc, 2 * (qb - qa), 2 * (qd - qc))]
    return blocks


def run_gpu(lib, blocks, nx0, ny0, d0, f, dt, bcs, steps=1, **opt):
    fo = lib.Forest(blocks, nx0, ny0, d0, d0, [(b.kind, b.value) for b in bcs], lib.default_options(**opt))
    t = {k: torch.tensor(v, dtype=torch.float64, device="cuda") for k, v in f.items()}
    infos = []
    for _ in range(steps):
        infos.append(fo.step(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], dt, check=False))
    torch.cuda.synchronize()
    xc, yc, lv = fo.centres()
    fo.close()
    return t["E"].cpu().numpy(), t["T"].cpu().numpy(), infos, (xc, yc, lv)


BCS = [O.BCSpec(O.DIRICHLET_FACE, 2e4), O.BCSpec(O.FREE_STREAM), O.BCSpec(O.FLUX_IN, 1e12), O.BCSpec(O.REFLECT)]


@pytest.mark.parametrize("nx0,ny0,bcs", [(8, 8, [O.BCSpec()] * 4), (16, 12, BCS), (64, 48, BCS)])
def test_forest_matches_oracle(lib, nx0, ny0, bcs):
    blocks = nested_patches(nx0, ny0)
    F = FF.build([FF.Block(*b) for b in blocks], 1e10, 1e10, nx0, ny0)
    f = fields_for(F.n, nx0)
    print(f"[forest] {nx0}x{ny0} base, {F.n} cells, levels {sorted(set(F.level))}", flush=True)
    ref = FF.step(F, f["E"], f["T"], f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], 1e4, bcs)
    E, T, infos, (xc, yc, lv) = run_gpu(lib, blocks, nx0, ny0, 1e10, f, 1e4, bcs, **PAR)
    print(infos[0]["inner_iters"], infos[0]["rel_resid"], rel_l2(E, ref.E), rel_l2(T, ref.T), flush=True)
    np.testing.assert_array_equal(lv, F.level)
    np.testing.assert_allclose(xc, F.xc, rtol=1e-15)
    np.testing.assert_allclose(yc, F.yc, rtol=1e-15)
    assert infos[0]["status"] == 0
    assert rel_l2(E, ref.E) < 1e-10 and rel_l2(T, ref.T) < 1e-10


def test_forest_three_steps(lib):
    nx0, ny0 = 32, 32
    blocks = nested_patches(nx0, ny0)
    F = FF.build([FF.Block(*b) for b in blocks], 1e10, 1e10, nx0, ny0)
    f = fields_for(F.n, 3)
    E, T = f["E"], f["T"]
    for _ in range(3):
        r = FF.step(F, E, T, f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], 1e4, BCS)
        E, T = r.E, r.T
    Eg, Tg, infos, _ = run_gpu(lib, blocks, nx0, ny0, 1e10, f, 1e4, BCS, steps=3, **PAR)
    assert all(i["status"] == 0 for i in infos)
    assert rel_l2(Eg, E) < 1e-10 and rel_l2(Tg, T) < 1e-10


def test_uniform_forest_equals_single_grid_step(lib):
    """Level-0 blocks tiling the 1024 x 1024 stretched recipe's first 96 x 80
    cells with uniform spacing: the forest step equals the single-grid step
    (same system; different solvers, both to 1e-12)."""
    prob = W.make_c1(nx=96, ny=80)
    prob.bc = [W.BC(W.BC_DIRICHLET_FACE, 2e4), W.BC(), W.BC(W.BC_FLUX_IN, 1e12), W.BC(W.BC_FREE_STREAM)]
    blocks = [(0, 0, 0, 48, 40), (0, 48, 0, 48, 40), (0, 0, 40, 96, 40)]
    F = FF.build([FF.Block(*b) for b in blocks], 1e10, 1e10, 96, 80)
    ci = np.rint(F.xc / 1e10 - 0.5).astype(int)
    cj = np.rint(F.yc / 1e10 - 0.5).astype(int)
    f = {k: np.ascontiguousarray(getattr(prob, k)[cj, ci]) for k in ("E", "T", "rho", "kappa_R", "kappa_P", "c_v")}
    bcs = O.bcs_from_problem(prob)
    E, T, infos, _ = run_gpu(lib, blocks, 96, 80, 1e10, f, prob.dt, bcs, **PAR)
    ctx = make_ctx(lib, prob, precision="fp64", rel_tol=1e-12, norm=1)
    t = to_dev(prob, torch)
    ctx.step(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, None)
    torch.cuda.synchronize()
    ctx.close()
    Eg, Tg = t["E"].cpu().numpy()[cj, ci], t["T"].cpu().numpy()[cj, ci]
    assert infos[0]["status"] == 0
    assert rel_l2(E, Eg) < 1e-10 and rel_l2(T, Tg) < 1e-10


def test_forest_errors(lib):
    with pytest.raises(lib.FLDError) as e:
        lib.Forest([(0, 0, 0, 4, 4), (0, 2, 2, 4, 4)], 8, 8, 1e10, 1e10)
    assert e.value.status == lib.FLD_EINVAL
    with pytest.raises(lib.FLDError):  # a level-2 block beside level-0 cells
        lib.Forest([(0, 0, 0, 4, 8), (2, 16, 0, 16, 32)], 8, 8, 1e10, 1e10)
    with pytest.raises(lib.FLDError):
        lib.Forest([(0, 0, 0, 8, 8)], 8, 8, 1e10, 1e10, options=lib.default_options(precision="mixed"))
    fo = lib.Forest([(0, 0, 0, 8, 8)], 8, 8, 1e10, 1e10)
    f = fields_for(64, 1)
    f["T"][5] = -1.0
    t = {k: torch.tensor(v, dtype=torch.float64, device="cuda") for k, v in f.items()}
    r = fo.step(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], 1e4, check=False)
    assert r["status"] == lib.FLD_ENONFINITE
    fo.close()
