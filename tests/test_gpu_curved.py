"""GPU parity on curved (multilinear) elements against the FP64 oracle,
through the C ABI: lattices whose vertices are moved by seeded noise
(+-10% of the spacing, periodic images moved together), each element with its
own orthonormalised basis, Nanson normals and area weights.

Bounds as on the affine lattices: residual and exact Jv 1e-12 relative
(the residual normalised by the larger of its total and volume parts), block
Jacobi 1e-11, one V-cycle 1e-9; the FP32 operator 1e-5 (and above 1e-10),
FP32 block factors 1e-4.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import DGOracle, NavierStokes, block_solve
from oracle.pmg import PMultigrid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300)


def make_curved(N, order, space, nq, flux="roe", mu=1e-2, seed=13, perturb=0.1):
    from paper_1809_00866_amd import DG
    mesh = synth.lattice_mesh(N, L=1.0, perturb=perturb, seed=seed)
    d = len(N)
    o = DGOracle(mesh, order, space, nq, NavierStokes(d, mu=mu, flux=flux))
    g = DG(mesh, order, basis=space, nq1d=nq, flux=flux, mu=mu)
    fld = synth.FreeStreamPlusModes(seed=seed) if d == 2 else synth.TaylorGreenStandIn(seed=seed, L=1.0)
    U = o.project(fld)
    U = U + 1e-2 * np.random.default_rng(seed).standard_normal(U.shape) * np.abs(U[:, :, :1])
    w = torch.tensor(o.to_flat(U), device="cuda")
    return mesh, o, g, U, w, fld


CASES = [
    ((3, 3), 2, "Q", 4, "roe"),
    ((3, 4), 2, "P", 4, "lf"),
    ((2, 2, 2), 1, "P", 2, "lf"),
    ((2, 3, 2), 2, "P", 3, "roe"),
    ((2, 2, 3), 3, "P", 4, "roe"),
    ((2, 2, 1), 4, "P", 5, "roe"),
]
IDS = [f"{len(c[0])}d-N{'x'.join(map(str, c[0]))}-{c[2]}{c[1]}-{c[4]}" for c in CASES]


@pytest.mark.parametrize("N,k,sp,nq,flux", CASES, ids=IDS)
def test_curved_residual_and_jvp_parity(N, k, sp, nq, flux):
    _say(f"curved residual/jvp {N} {sp}{k} {flux}")
    mesh, o, g, U, w, fld = make_curved(N, k, sp, nq, flux)
    R, Rv = o.residual(U, return_parts=True)
    Rg = g.residual(w).cpu().numpy()
    err = np.linalg.norm(Rg - o.to_flat(R)) / max(np.linalg.norm(R), np.linalg.norm(Rv))
    assert err <= 1e-12, err
    V = np.random.default_rng(3).standard_normal(U.shape)
    v = torch.tensor(o.to_flat(V), device="cuda")
    ref = o.to_flat(o.jvp(U, V) + 2.0 * V)
    assert rel(g.jvp(w, v, shift=2.0).cpu().numpy(), ref) <= 1e-12
    assert rel(g.jvp(w, v, mode="stab").cpu().numpy(), o.to_flat(o.stab_jvp(U, V))) <= 1e-12
    g.close()


def test_curved_results_are_bitwise_repeatable():
    """The FP64 face kernel sums the two sides' gradient traces by two LDS
    atomic adds in either order (a + b both ways): repeated residuals and Jv
    on a curved P4 mesh of several tiles are equal bit for bit, FP64 and FP32."""
    _say("curved repeatability")
    mesh, o, g, U, w, fld = make_curved((4, 3, 3), 4, "P", 5, "roe")
    v = torch.randn(g.ndof, dtype=torch.float64, device="cuda", generator=torch.Generator(device="cuda").manual_seed(7))
    for mode in ("exact", "exact_fp32"):
        a, b = g.jvp(w, v, shift=1.5, mode=mode), g.jvp(w, v, shift=1.5, mode=mode)
        assert torch.equal(a, b), mode
    assert torch.equal(g.residual(w), g.residual(w))
    g.close()


def test_curved_points_projection_and_free_stream():
    _say("curved points / projection / free stream")
    mesh, o, g, U, w, fld = make_curved((2, 3, 2), 3, "P", 4)
    xyz = g.volume_points().cpu().numpy()                      # [dim, nq, ne]
    et = o.elem_tables(np.arange(o.ne))
    assert np.abs(np.moveaxis(xyz, 0, -1).transpose(1, 0, 2) - et["x"]).max() < 1e-13
    assert rel(g.project_field(fld).cpu().numpy(), o.to_flat(o.project(fld))) <= 1e-13
    const = lambda x: np.broadcast_to(np.array([1.0, 0.3, -0.2, 0.1, 2.5]), x.shape[:-1] + (5,))
    wc = g.project_field(const)
    r = g.residual(wc).cpu().numpy()
    assert np.abs(r).max() <= 1e-12 * np.abs(wc.cpu().numpy()).max()
    assert g.max_wave_speed(w) == pytest.approx(
        float(np.max(o.phys.max_wave_speed(np.einsum("eqb,ecb->eqc", et["phi"], U)))), rel=1e-12)
    g.close()


def test_curved_block_jacobi_and_vcycle():
    _say("curved block Jacobi and V-cycle")
    mesh, o, g, U, w, fld = make_curved((2, 2, 2), 2, "P", 3)
    shift = 8.0
    r = np.random.default_rng(5).standard_normal(U.shape)
    rt = torch.tensor(o.to_flat(r), device="cuda")
    D = o.block_diagonal(U, shift=shift)
    g.block_setup(w, shift)
    z = g.block_apply(rt).cpu().numpy()
    assert rel(z, o.to_flat(block_solve(D, r.reshape(o.ne, -1)).reshape(U.shape))) <= 1e-11
    mg = PMultigrid(o, U, shift, (2, 1), (3, 10))
    g.mg_setup(w, shift, (2, 1), (3, 10), storage="fp64", use_graph=True)
    z_o = o.to_flat(mg.apply(r))
    assert rel(g.mg_apply(rt).cpu().numpy(), z_o) <= 1e-9
    b = torch.tensor(o.to_flat(np.random.default_rng(6).standard_normal(U.shape)), device="cuda")
    x, st = g.fgmres(w, shift, b, rtol=1e-10, max_iter=500, precond="mg")
    assert st["converged"] == 1
    X = o.from_flat(x.cpu().numpy())
    res = np.linalg.norm(o.to_flat(o.operator(U, X, shift)) - b.cpu().numpy()) / b.norm().item()
    assert res <= 1e-9
    g.close()


@pytest.mark.parametrize("N,k,sp,nq", [((3, 2, 3), 3, "P", 4), ((3, 4), 2, "P", 4)], ids=["3d-P3", "2d-P2"])
def test_curved_element_local_probing_matches_coloured_bitwise(N, k, sp, nq):
    """On curved elements too, probing the diagonal blocks element by element
    (the face kernel run once per side, the second run writing the jump and
    flux records that the volume kernel reads on the -p faces) gives the
    coloured probe's blocks bit for bit (Sec. 2.3): FP64 and FP32 probing in
    the block setup and in the p-multigrid setup's fine blocks."""
    _say(f"curved local vs coloured probing {N} {sp}{k}")
    mesh, o, g, U, w, fld = make_curved(N, k, sp, nq)
    g.set_tuning("fixed")
    shift = 8.0
    r = torch.randn(g.ndof, dtype=torch.float64, device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    out = {}
    for mode in ("coloured", "auto"):
        g.set_block_probing(mode)
        for storage in ("fp64", "fp32"):
            g.block_setup(w, shift, storage=storage)
            out[mode, storage] = g.block_apply(r).clone()
        for fp in ("fp64", "fp32"):
            g.mg_setup(w, shift, (k, 1), (3, 10), storage="fp32", use_graph=True, fine_precision=fp)
            out[mode, "mg", fp] = g.mg_apply(r).clone()
    for key, z in out.items():
        if key[0] == "auto":
            assert torch.isfinite(z).all(), key
            assert torch.equal(z, out[("coloured",) + key[1:]]), key
    g.close()


@pytest.mark.parametrize("N,k,sp,nq,flux", [CASES[0], CASES[3], CASES[5]], ids=[IDS[0], IDS[3], IDS[5]])
def test_curved_fp32_operator_error_against_the_oracle(N, k, sp, nq, flux):
    """The curved kernels in FP32 (tables, contractions, pointwise fluxes;
    FP64 inputs and outputs): a reduced-precision operator for the
    preconditioners, within 1e-5 of the FP64 oracle and genuinely FP32."""
    _say(f"curved fp32 operator {N} {sp}{k} {flux}")
    mesh, o, g, U, w, fld = make_curved(N, k, sp, nq, flux)
    R, Rv = o.residual(U, return_parts=True)
    r32 = g.residual(w, precision="fp32").cpu().numpy()
    err_r = np.linalg.norm(r32 - o.to_flat(R)) / max(np.linalg.norm(R), np.linalg.norm(Rv))
    V = np.random.default_rng(866).standard_normal(U.shape)
    v = torch.tensor(o.to_flat(V), device="cuda")
    err_j = rel(g.jvp(w, v, shift=3.0, mode="exact_fp32").cpu().numpy(), o.to_flat(o.jvp(U, V) + 3.0 * V))
    _say(f"  fp32 residual error {err_r:.2e}, Jv error {err_j:.2e}")
    assert 1e-10 < err_r <= 1e-5 and 1e-10 < err_j <= 1e-5
    g.close()


def test_curved_fp32_probing_and_smoothing():
    """Block Jacobi probed with the FP32 curved operator (FP32 factors) and
    the V-cycle with FP32 fine-level smoothing: both precondition an FGMRES
    solve whose FP64 true residual reaches the tolerance."""
    _say("curved fp32 probing and smoothing")
    mesh, o, g, U, w, fld = make_curved((2, 2, 2), 2, "P", 3)
    shift = 8.0
    r = np.random.default_rng(5).standard_normal(U.shape)
    rt = torch.tensor(o.to_flat(r), device="cuda")
    D = o.block_diagonal(U, shift=shift)
    g.block_setup(w, shift, storage="fp32")
    z = g.block_apply(rt).cpu().numpy()
    assert rel(z, o.to_flat(block_solve(D, r.reshape(o.ne, -1)).reshape(U.shape))) <= 1e-4
    b = torch.tensor(o.to_flat(np.random.default_rng(6).standard_normal(U.shape)), device="cuda")
    for precond in ("bj", "mg"):
        if precond == "mg":
            g.mg_setup(w, shift, (2, 1), (3, 10), storage="fp32", use_graph=True, fine_precision="fp32")
        x, st = g.fgmres(w, shift, b, rtol=1e-10, max_iter=500, precond=precond)
        assert st["converged"] == 1, precond
        X = o.from_flat(x.cpu().numpy())
        res = np.linalg.norm(o.to_flat(o.operator(U, X, shift)) - b.cpu().numpy()) / b.norm().item()
        assert res <= 1e-9, (precond, res)
    g.close()


def test_curved_rescaled_inherited_hierarchy():
    """App. A on curved elements: the stabilisation part of every inherited
    coarse operator rescaled level by level (1e-12 per level) and the
    V-cycle on them (1e-9), against the oracle."""
    _say("curved rescaled hierarchy")
    mesh, o, g, U, w, fld = make_curved((2, 2, 2), 2, "P", 3, mu=5e-2)
    shift, orders, iters = 8.0, (2, 1), (3, 10)
    mg = PMultigrid(o, U, shift, orders, iters, rescale=True)
    g.mg_setup(w, shift, orders, iters, storage="fp64", use_graph=True, rescale=True)
    rng = np.random.default_rng(24)
    for l in range(1, mg.L + 1):
        X = rng.standard_normal((o.ne, o.nvar, mg.nbs[l]))
        y_o = (mg.A[l] @ X.reshape(-1)).reshape(X.shape)
        xg = torch.tensor(np.ascontiguousarray(X.transpose(1, 2, 0)).reshape(-1), device="cuda")
        y_g = g.mg_level_apply(l, xg).cpu().numpy().reshape(o.nvar, mg.nbs[l], o.ne).transpose(2, 0, 1)
        assert np.linalg.norm(y_g - y_o) <= 1e-12 * np.linalg.norm(y_o), (l, np.linalg.norm(y_g - y_o))
    R = rng.standard_normal(U.shape)
    z_o = o.to_flat(mg.apply(R))
    assert rel(g.mg_apply(torch.tensor(o.to_flat(R), device="cuda")).cpu().numpy(), z_o) <= 1e-9
    g.close()


def test_curved_fd_jvp_and_rosenbrock_step():
    """On a curved mesh: the finite-difference Jv (eq. epsdef) within 1e-6 of
    the exact tangent, and one ROS2 step (each stage solved by FGMRES to 1e-12)
    within 1e-10 of the oracle's dense step, relative to the increment."""
    from oracle import rosenbrock as ros
    _say("curved fd jvp and rosenbrock step")
    mesh, o, g, U, w, fld = make_curved((2, 1, 2), 1, "P", 2)
    V = np.random.default_rng(9).standard_normal(U.shape)
    v = torch.tensor(o.to_flat(V), device="cuda")
    assert rel(g.jvp(w, v, mode="fd").cpu().numpy(), o.to_flat(o.jvp(U, V))) <= 1e-6
    coeffs, dt = ros.ros2(), 0.05
    U1 = ros.dg_step(o, U, dt, coeffs)
    g.block_setup(w, 1.0 / (coeffs["gamma"] * dt))
    w1, st = g.rosenbrock_step(w, dt, coeffs, rtol=1e-12, max_iter=500, precond="bj")
    assert st["converged"] == 1
    d_o = o.to_flat(U1) - o.to_flat(U)
    d_g = w1.cpu().numpy() - o.to_flat(U)
    assert np.linalg.norm(d_g - d_o) <= 1e-10 * np.linalg.norm(d_o)
    g.close()
