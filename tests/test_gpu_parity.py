"""GPU parity: the HIP library through the C ABI against the FP64 oracle.

Tolerances (relative 2-norms): residual 1e-12 of max(|R|, |R_volume|), exact
Jv 1e-12, FD Jv 1e-6 (the FD quotient amplifies round-off by 1/Delta),
projection 1e-13, block apply 1e-11 (FP64) / 1e-4 (FP32 factors) / the
entrywise BF16 rounding bound 2^-8 |D^-1||r| (BF16 factors), solves
checked on the true residual with the oracle operator.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import DGOracle, NavierStokes, block_solve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_case(N, order, space, nq, flux="roe", mu=1e-2, seed=11, noise=1e-2):
    from paper_1809_00866_amd import DG
    mesh = synth.lattice_mesh(N, L=1.0)
    d = len(N)
    o = DGOracle(mesh, order, space, nq, NavierStokes(d, mu=mu, flux=flux))
    g = DG(mesh, order, basis=space, nq1d=nq, flux=flux, mu=mu)
    fld = synth.FreeStreamPlusModes(seed=seed) if d == 2 else synth.TaylorGreenStandIn(seed=seed, L=1.0)
    U = o.project(fld)
    rng = np.random.default_rng(seed)
    U = U + noise * rng.standard_normal(U.shape) * np.abs(U[:, :, :1])
    w = torch.tensor(o.to_flat(U), device="cuda")
    return o, g, U, w


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


CASES = [
    ((4, 4), 2, "Q", 4, "roe"),       # the 2D Q2 discretisation
    ((3, 5), 2, "P", 4, "lf"),        # 2D P2, Lax-Friedrichs, odd sizes
    ((2, 3, 5), 3, "P", 4, "roe"),    # 3D P3, ragged tiles
    ((3, 2, 2), 4, "P", 5, "roe"),    # 3D P4
    ((2, 2, 2), 1, "P", 2, "lf"),     # 3D P1
    ((3, 3, 2), 2, "P", 3, "roe"),    # 3D P2
    ((1, 1, 1), 3, "P", 4, "roe"),    # one periodic element: its own neighbour
]
IDS = [f"{len(c[0])}d-N{'x'.join(map(str, c[0]))}-{c[2]}{c[1]}-{c[4]}" for c in CASES]


@pytest.mark.parametrize("N,k,sp,nq,flux", CASES, ids=IDS)
def test_residual_parity(N, k, sp, nq, flux):
    _say(f"residual parity {N} {sp}{k} {flux}")
    o, g, U, w = make_case(N, k, sp, nq, flux)
    R, Rv = o.residual(U, return_parts=True)
    Rg = g.residual(w).cpu().numpy()
    err = np.linalg.norm(Rg - o.to_flat(R)) / max(np.linalg.norm(R), np.linalg.norm(Rv))
    assert err <= 1e-12, err


@pytest.mark.parametrize("N,k,sp,nq,flux", CASES, ids=IDS)
def test_jvp_exact_parity(N, k, sp, nq, flux):
    _say(f"jvp parity {N} {sp}{k} {flux}")
    o, g, U, w = make_case(N, k, sp, nq, flux)
    V = np.random.default_rng(866).standard_normal(U.shape)
    v = torch.tensor(o.to_flat(V), device="cuda")
    Jv = o.jvp(U, V)
    for shift in (0.0, 37.5):
        out = g.jvp(w, v, shift=shift, mode="exact").cpu().numpy()
        assert rel(out, o.to_flat(Jv + shift * V)) <= 1e-12


@pytest.mark.parametrize("N,k,sp,nq,flux", [CASES[0], CASES[2]], ids=[IDS[0], IDS[2]])
def test_jvp_fd_parity(N, k, sp, nq, flux):
    _say(f"fd jvp parity {N}")
    o, g, U, w = make_case(N, k, sp, nq, flux)
    V = np.random.default_rng(3).standard_normal(U.shape)
    v = torch.tensor(o.to_flat(V), device="cuda")
    fd_o = o.to_flat(o.jvp_fd(U, V))
    ex_o = o.to_flat(o.jvp(U, V))
    fd_g = g.jvp(w, v, mode="fd").cpu().numpy()
    assert rel(fd_g, fd_o) <= 1e-6
    assert rel(fd_g, ex_o) <= 1e-5
    r_w = g.residual(w)
    fd_g2 = g.jvp(w, v, mode="fd", r_w=r_w).cpu().numpy()
    assert np.array_equal(fd_g, fd_g2)
    zero = torch.zeros_like(v)
    assert torch.count_nonzero(g.jvp(w, zero, shift=2.0, mode="fd")) == 0


def test_projection_and_points():
    _say("projection parity")
    o, g, U, w = make_case((3, 2, 4), 3, "P", 4)
    xyz = g.volume_points().cpu().numpy()          # [dim, nq, ne]
    et = o.elem_tables(np.arange(o.ne))
    assert np.abs(np.moveaxis(xyz, 0, -1).transpose(1, 0, 2) - et["x"]).max() < 1e-14
    fld = synth.TaylorGreenStandIn(seed=5, L=1.0)
    wg = g.project_field(fld).cpu().numpy()
    assert rel(wg, o.to_flat(o.project(fld))) <= 1e-13


@pytest.mark.parametrize("N,k,sp,nq,flux", [CASES[0], CASES[2], CASES[3], CASES[6]],
                         ids=[IDS[0], IDS[2], IDS[3], IDS[6]])
def test_block_jacobi_parity(N, k, sp, nq, flux):
    _say(f"block parity {N} {sp}{k}")
    o, g, U, w = make_case(N, k, sp, nq, flux)
    shift = 25.0
    D = o.block_diagonal(U, shift=shift)
    r = np.random.default_rng(4).standard_normal(U.shape)
    z_o = block_solve(D, r.reshape(o.ne, -1)).reshape(U.shape)
    rt = torch.tensor(o.to_flat(r), device="cuda")
    g.block_setup(w, shift, storage="fp64")
    z_g = g.block_apply(rt).cpu().numpy()
    assert rel(z_g, o.to_flat(z_o)) <= 1e-11
    if o.nb * o.nvar * o.nb * o.nvar * 4 <= 150 * 1024:
        g.block_setup(w, shift, storage="fp32")
        z_g32 = g.block_apply(rt).cpu().numpy()
        assert rel(z_g32, o.to_flat(z_o)) <= 1e-4
        # BF16 factors: every stored entry of D^-1 carries a relative rounding
        # error <= 2^-9, so |z - z_exact| <= 2^-9 |D^-1| |r| entrywise, plus the
        # FP32 elimination and accumulation error (well below 2^-9 here).
        g.block_setup(w, shift, storage="bf16")
        z_b = o.from_flat(g.block_apply(rt).cpu().numpy()).reshape(o.ne, -1)
        Dinv = np.linalg.inv(D)
        bound = np.einsum("eij,ej->ei", np.abs(Dinv), np.abs(r.reshape(o.ne, -1)))
        err = np.abs(z_b - z_o.reshape(o.ne, -1))
        assert np.all(err <= 2.0 ** -8 * bound + 1e-12), (err / bound).max()


PROBE_CASES = [((4, 4, 3), 4, 5), ((5, 2, 3), 3, 4), ((3, 3, 2), 2, 3)]


@pytest.mark.parametrize("N,k,nq", PROBE_CASES, ids=[f"N{'x'.join(map(str, c[0]))}-P{c[1]}" for c in PROBE_CASES])
def test_element_local_probing_matches_coloured_bitwise(N, k, nq):
    """Element-local probing of the diagonal blocks (every element perturbed at
    once, the face kernel run once per side) gives the coloured probe's blocks
    bit for bit (Sec. 2.3: both read the exact Jacobian's diagonal blocks, the
    local one with the other side's tangent zero instead of a zero input):
    FP64 and FP32 probing in the block setup, the FP32 and BF16-contraction
    operators in the p-multigrid setup's fine blocks; several tiles, ragged
    last tiles, a direction of two elements (both neighbours the same
    element)."""
    _say(f"local vs coloured probing {N} P{k}")
    o, g, U, w = make_case(N, k, "P", nq)
    g.set_tuning("fixed")  # the same launch shapes for both setups
    shift = 25.0
    r = torch.randn(g.ndof, dtype=torch.float64, device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    out = {}
    for mode in ("coloured", "auto"):
        g.set_block_probing(mode)
        for storage in ("fp64", "fp32"):
            g.block_setup(w, shift, storage=storage)
            out[mode, storage] = g.block_apply(r).clone()
        for fp in ("fp64", "fp32", "bf16"):
            g.mg_setup(w, shift, [k, 1], [2, 4], storage="fp32", fine_precision=fp)
            out[mode, "mg", fp] = g.mg_apply(r).clone()
    for key, z in out.items():
        if key[0] == "auto":
            assert torch.isfinite(z).all(), key
            assert torch.equal(z, out[("coloured",) + key[1:]]), key
    assert g.lib.dg_set_block_probing(g.ctx, 7) == -1  # DG_ERR_ARG: unknown mode
    g.close()


def test_block_apply_before_setup_is_state_error():
    from paper_1809_00866_amd._lib import DGError
    o, g, U, w = make_case((2, 2, 2), 1, "P", 2)
    with pytest.raises(DGError) as ei:
        g.block_apply(w)
    assert ei.value.status == -4


@pytest.mark.parametrize("precond", ["bj", "none"])
def test_fgmres_true_residual_with_oracle_operator(precond):
    _say(f"fgmres {precond}")
    o, g, U, w = make_case((3, 3, 3), 2, "P", 3)
    shift = 40.0
    B = np.random.default_rng(5).standard_normal(U.shape)
    b = torch.tensor(o.to_flat(B), device="cuda")
    if precond == "bj":
        g.block_setup(w, shift)
    x, st = g.fgmres(w, shift, b, restart=30, rtol=1e-10, max_iter=2000, precond=precond)
    assert st["converged"] == 1 and st["rel_res_true"] <= 1e-10
    X = o.from_flat(x.cpu().numpy())
    res = np.linalg.norm(o.to_flat(o.operator(U, X, shift)) - o.to_flat(B)) / np.linalg.norm(B)
    assert res <= 1e-9


def test_fgmres_modified_gram_schmidt():
    """orth="mgs": the same Krylov spaces as CGS2 (iteration counts within one),
    the true residual checked with the oracle operator."""
    _say("fgmres mgs")
    o, g, U, w = make_case((3, 3, 3), 2, "P", 3)
    shift = 40.0
    B = np.random.default_rng(7).standard_normal(U.shape)
    b = torch.tensor(o.to_flat(B), device="cuda")
    g.block_setup(w, shift)
    x1, s1 = g.fgmres(w, shift, b, restart=20, rtol=1e-10, max_iter=2000, precond="bj", orth="mgs")
    x2, s2 = g.fgmres(w, shift, b, restart=20, rtol=1e-10, max_iter=2000, precond="bj", orth="cgs2")
    assert s1["converged"] == 1 and abs(s1["iters"] - s2["iters"]) <= 1
    X = o.from_flat(x1.cpu().numpy())
    res = np.linalg.norm(o.to_flat(o.operator(U, X, shift)) - o.to_flat(B)) / np.linalg.norm(B)
    assert res <= 1e-9
    assert rel(x1.cpu().numpy(), x2.cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_fgmres_reduced_precision_blocks_reach_fp64_tolerance(storage):
    """Reduced-precision block factors change only the preconditioner: the FP64
    flexible outer iteration still reaches 1e-10 on the true residual."""
    _say(f"fgmres {storage} blocks")
    o, g, U, w = make_case((3, 3, 3), 2, "P", 3)
    shift = 40.0
    B = np.random.default_rng(5).standard_normal(U.shape)
    b = torch.tensor(o.to_flat(B), device="cuda")
    g.block_setup(w, shift, storage="fp64")
    _, st64 = g.fgmres(w, shift, b, restart=30, rtol=1e-10, max_iter=2000, precond="bj")
    g.block_setup(w, shift, storage=storage)
    x, st = g.fgmres(w, shift, b, restart=30, rtol=1e-10, max_iter=2000, precond="bj")
    assert st["converged"] == 1 and st["rel_res_true"] <= 1e-10
    assert st["iters"] <= st64["iters"] + 10
    X = o.from_flat(x.cpu().numpy())
    res = np.linalg.norm(o.to_flat(o.operator(U, X, shift)) - o.to_flat(B)) / np.linalg.norm(B)
    assert res <= 1e-9


def test_fgmres_edge_cases():
    _say("fgmres edge cases")
    o, g, U, w = make_case((2, 2, 2), 2, "P", 3)
    b = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    x, st = g.fgmres(w, 10.0, b, x=torch.ones_like(b), precond="none")
    assert st["converged"] == 1 and st["iters"] == 0 and torch.count_nonzero(x) == 0
    b = torch.randn(g.ndof, dtype=torch.float64, device="cuda")
    x, st = g.fgmres(w, 10.0, b, max_iter=1, rtol=1e-14, precond="none")
    assert st["converged"] == 0 and st["iters"] == 1
    from paper_1809_00866_amd._lib import DGError
    bad = b.clone()
    bad[3] = float("nan")
    with pytest.raises(DGError) as ei:
        g.fgmres(w, 10.0, bad, precond="none")
    assert ei.value.status == -6


def test_determinism():
    o, g, U, w = make_case((2, 3, 5), 3, "P", 4)
    v = torch.randn(g.ndof, dtype=torch.float64, device="cuda")
    a, b2 = g.residual(w), g.residual(w)
    assert torch.equal(a, b2)
    assert torch.equal(g.jvp(w, v), g.jvp(w, v))


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_full_size_sampled(name):
    """Full-size workloads in the benchmark's launch configuration; the oracle
    checks sampled elements (cfg1: all 256 elements)."""
    from paper_1809_00866_amd import DG
    _say(f"full-size sampled {name}")
    cfg, mesh, fld = synth.preset(name)
    d = cfg["dim"]
    o = DGOracle(mesh, cfg["order"], cfg["space"], cfg["nq1d"], NavierStokes(d, mu=cfg["mu"], flux="roe"))
    g = DG(mesh, cfg["order"], basis=cfg["space"], nq1d=cfg["nq1d"], flux="roe", mu=cfg["mu"])
    U = o.project(fld)
    w = torch.tensor(o.to_flat(U), device="cuda")
    v = torch.tensor(synth.random_vector(g.ndof, cfg["v_seed"]), device="cuda")
    V = o.from_flat(v.cpu().numpy())
    Rg = o.from_flat(g.residual(w).cpu().numpy())
    Jg = o.from_flat(g.jvp(w, v).cpu().numpy())
    rng = np.random.default_rng(0)
    sample = np.arange(o.ne) if o.ne <= 256 else np.unique(np.concatenate(
        [[0, o.ne - 1], rng.choice(o.ne, 14, replace=False)]))
    R, Rv = o.residual(U, elems=sample, return_parts=True)
    scale = max(np.linalg.norm(R), np.linalg.norm(Rv))
    assert np.linalg.norm(Rg[sample] - R) <= 1e-12 * scale
    J = o.jvp(U, V, elems=sample)
    assert np.linalg.norm(Jg[sample] - J) <= 1e-12 * np.linalg.norm(J)


@pytest.mark.parametrize("N,k,sp,nq,flux", [CASES[0], CASES[2], CASES[3], CASES[4]],
                         ids=[IDS[0], IDS[2], IDS[3], IDS[4]])
def test_stabilisation_jvp_parity(N, k, sp, nq, flux):
    """The BR2 stabilisation part of the Jacobian (jvp mode "stab") against the
    oracle's complex-step derivative through the face lifting term, 1e-12."""
    _say(f"stabilisation jvp {N} {sp}{k}")
    o, g, U, w = make_case(N, k, sp, nq, flux)
    V = np.random.default_rng(44).standard_normal(U.shape)
    v = torch.tensor(o.to_flat(V), device="cuda")
    ref = o.to_flat(o.stab_jvp(U, V))
    out = g.jvp(w, v, mode="stab").cpu().numpy()
    assert rel(out, ref) <= 1e-12, rel(out, ref)
    out2 = g.jvp(w, v, shift=2.5, mode="stab").cpu().numpy()
    assert rel(out2, ref + 2.5 * o.to_flat(V)) <= 1e-12


@pytest.mark.parametrize("N,k,nq", [((2, 3, 5), 3, 4), ((3, 2, 3), 4, 5), ((3, 3, 2), 2, 3)],
                         ids=["P3", "P4", "P2"])
def test_mfma_and_reference_kernels_agree(N, k, nq, monkeypatch):
    """The MFMA kernels and the reference kernels compute the same residual and Jv."""
    from paper_1809_00866_amd import DG
    _say(f"mfma vs reference {N} P{k}")
    mesh = synth.lattice_mesh(N, L=1.0)
    fld = synth.TaylorGreenStandIn(seed=12, L=1.0)
    monkeypatch.setenv("DG_KERNEL_VARIANT", "reference")
    gr = DG(mesh, k, nq1d=nq, mu=1e-2)
    monkeypatch.setenv("DG_KERNEL_VARIANT", "mfma")
    gm = DG(mesh, k, nq1d=nq, mu=1e-2)
    w = gr.project_field(fld)
    v = torch.randn(gr.ndof, dtype=torch.float64, device="cuda")
    r0, r1 = gr.residual(w), gm.residual(w)
    assert (r0 - r1).norm() <= 1e-13 * r0.norm() * 1e2
    j0, j1 = gr.jvp(w, v, shift=1.5), gm.jvp(w, v, shift=1.5)
    assert (j0 - j1).norm() <= 1e-13 * j0.norm() * 1e2


@pytest.mark.parametrize("N,k,sp,nq,flux", [CASES[2], CASES[3], CASES[5]], ids=[IDS[2], IDS[3], IDS[5]])
def test_fp32_operator_error_against_the_oracle(N, k, sp, nq, flux):
    """FP32 contractions and pointwise arithmetic: a reduced-precision operator
    for preconditioners.  Its error against the FP64 oracle is bounded by 1e-5
    (relative, residual normalised like the FP64 test) and is genuinely FP32
    (above 1e-10)."""
    _say(f"fp32 operator {N} {sp}{k}")
    o, g, U, w = make_case(N, k, sp, nq, flux)
    R, Rv = o.residual(U, return_parts=True)
    r32 = g.residual(w, precision="fp32").cpu().numpy()
    err_r = np.linalg.norm(r32 - o.to_flat(R)) / max(np.linalg.norm(R), np.linalg.norm(Rv))
    V = np.random.default_rng(866).standard_normal(U.shape)
    v = torch.tensor(o.to_flat(V), device="cuda")
    ref = o.to_flat(o.jvp(U, V) + 3.0 * V)
    j32 = g.jvp(w, v, shift=3.0, mode="exact_fp32").cpu().numpy()
    err_j = rel(j32, ref)
    _say(f"  fp32 residual error {err_r:.2e}, Jv error {err_j:.2e}")
    assert 1e-10 < err_r <= 1e-5 and 1e-10 < err_j <= 1e-5


@pytest.mark.parametrize("N,k,sp,nq,flux", [CASES[2], CASES[3], CASES[5]], ids=[IDS[2], IDS[3], IDS[5]])
def test_bf16_contraction_operator_error_against_the_oracle(N, k, sp, nq, flux):
    """BF16 contractions (BF16 operands, FP32 accumulation) with FP32 pointwise
    fluxes: error against the FP64 oracle within the 3e-2 bound for BF16
    contractions, measured and printed, and genuinely BF16 (above 1e-5)."""
    _say(f"bf16 operator {N} {sp}{k}")
    o, g, U, w = make_case(N, k, sp, nq, flux)
    R, Rv = o.residual(U, return_parts=True)
    rb = g.residual(w, precision="bf16").cpu().numpy()
    err_r = np.linalg.norm(rb - o.to_flat(R)) / max(np.linalg.norm(R), np.linalg.norm(Rv))
    V = np.random.default_rng(866).standard_normal(U.shape)
    v = torch.tensor(o.to_flat(V), device="cuda")
    ref = o.to_flat(o.jvp(U, V) + 3.0 * V)
    jb = g.jvp(w, v, shift=3.0, mode="exact_bf16").cpu().numpy()
    err_j = rel(jb, ref)
    ref0 = o.to_flat(o.jvp(U, V))
    err_j0 = rel(g.jvp(w, v, mode="exact_bf16").cpu().numpy(), ref0)
    _say(f"  bf16 residual error {err_r:.2e}, Jv error {err_j:.2e} (shift 3), {err_j0:.2e} (no shift)")
    assert 1e-5 < err_r <= 3e-2 and err_j <= 3e-2 and 1e-5 < err_j0 <= 3e-2


def test_fp32_operator_rejects_configurations_without_mfma_kernels():
    from paper_1809_00866_amd._lib import DGError
    o, g, U, w = make_case((4, 4), 2, "Q", 4)
    with pytest.raises(DGError) as ei:
        g.residual(w, precision="fp32")
    assert ei.value.status == -1
    with pytest.raises(DGError) as ei:
        g.residual(w, precision="bf16")
    assert ei.value.status == -1


@pytest.mark.parametrize("check_every", [1, 4, 7])
def test_fgmres_check_every_and_setup_time(check_every):
    """Convergence tested every check_every iterations (the GPU runs ahead,
    iterations past the converged one are discarded): the same iterations
    and solution bits as checking every iteration, the true residual
    re-checked with the oracle operator; ms_setup reports the block setup."""
    from paper_1809_00866_amd import DG
    mesh = synth.lattice_mesh((3, 3, 2), L=1.0)
    o = DGOracle(mesh, 3, "P", 4, NavierStokes(3, mu=1e-2))
    U = o.project(synth.TaylorGreenStandIn(seed=2, L=1.0))
    g = DG(mesh, 3, nq1d=4, mu=1e-2)
    w = torch.tensor(o.to_flat(U), device="cuda")
    shift = 20.0  # 99 block-Jacobi FGMRES(12) iterations to 1e-10 (the oracle's count)
    g.block_setup(w, shift, storage="fp64")
    B = np.random.default_rng(3).standard_normal(U.shape)
    b = torch.tensor(o.to_flat(B), device="cuda")
    x1, s1 = g.fgmres(w, shift, b, restart=12, rtol=1e-10, max_iter=400, precond="bj")
    xk, sk = g.fgmres(w, shift, b, restart=12, rtol=1e-10, max_iter=400, precond="bj", check_every=check_every)
    assert s1["converged"] == 1 and sk["converged"] == 1
    # the stop is found at the same column and the columns enqueued past it
    # are discarded: the same iterations and the same solution bits
    assert sk["iters"] == s1["iters"] and sk["restarts"] == s1["restarts"]
    assert torch.equal(xk, x1)
    assert sk["rel_res_true"] <= 1e-10
    X = o.from_flat(xk.cpu().numpy())
    res = np.linalg.norm(o.to_flat(o.operator(U, X, shift)) - o.to_flat(B)) / np.linalg.norm(B)
    assert res <= 1e-9
    assert sk["ms_setup"] > 0.0 and s1["ms_setup"] == sk["ms_setup"]
    g.close()
