"""GPU tests of the launch-shape autotuner and of every launch shape it can
choose, through the C ABI.

* MFMA occupancy (waves per SIMD of the face and volume kernels) and the
  volume kernel forming the corrected gradients itself: every variant
  computes the same bits as the default, residual and Jv, FP64, FP32 and
  BF16 operators, P2-P4 on a lattice of several 16-element tiles with a
  ragged tail, and at P4 24^3 (the solve workload's launch shape).
* Block-inverse apply shapes (one lane per row, 16-byte column loads with
  64-512 threads and 1-4 elements per workgroup): FP64 factors against the
  oracle's block solves (1e-12), FP32 / BF16 factors against the default
  shape (the same products summed in another order).
* Block-sparse coarse-operator apply shapes (workgroup size, rows per thread,
  column slices): the inherited P2 and P1 operators of a P3/P2/P1 hierarchy
  against the oracle's Galerkin operators (eq. GalProj, 1e-12), and one
  V-cycle with every coarse shape pinned against the oracle's V-cycle (Alg.
  vcic, 1e-9), the captured graph re-captured after each change; every shape
  of the FP32 copies the cycle applies with FP32 storage against the built-in
  one (1e-5).
* The tuned set-up (DG_TUNE_AUTO) against the fixed one: bitwise equal
  operator, block apply within 1e-13, V-cycle within 1e-10, and the report.
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


def _flat(X):
    return np.ascontiguousarray(np.transpose(X, (1, 2, 0))).reshape(-1)


def _unflat(x, ne, nv, nb):
    return np.ascontiguousarray(np.asarray(x).reshape(nv, nb, ne).transpose(2, 0, 1))


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300)


APPLY_SHAPES = [("row", 64, e) for e in (1, 2, 4, 8)] + [("vec", 64, e) for e in (1, 2, 4)] + \
    [("vec", t, 1) for t in (128, 256, 512)]
BSR_SHAPES = [(bs, rpt, cs) for bs in (256, 512, 1024) for rpt in (0, 1, 2, 4) for cs in (1, 2, 4, 8)]


def bsr_fits(bs, rpt, cs, m, elem, nf=6):
    """The launch predicate of the block-sparse apply, written out."""
    widest = 8 if elem == 2 and m % 8 == 0 else 4 if elem <= 4 and m % 4 == 0 else 2 if m % 2 == 0 else 1
    r = rpt or widest
    if r not in (1, 2) and not (r == 4 and elem <= 4) and not (r == 8 and elem == 2):
        return False
    return m % r == 0 and bs >= cs * (m // r) and ((nf + 1) * m + cs * m) * 8 <= 65536


def _state(mesh, k, nq, seed=3):
    o = DGOracle(mesh, k, "P", nq, NavierStokes(3, mu=1e-2))
    U = o.project(synth.TaylorGreenStandIn(seed=seed, L=1.0))
    U = U + 1e-2 * np.random.default_rng(seed).standard_normal(U.shape) * np.abs(U[:, :, :1])
    return o, U


@pytest.mark.parametrize("k,nq", [(2, 3), (3, 4), (4, 5)], ids=["P2", "P3", "P4"])
def test_every_fine_shape_computes_the_same_bits(k, nq):
    from paper_1809_00866_amd import DG
    from paper_1809_00866_amd._lib import DGError
    _say(f"occupancy variants P{k}")
    mesh = synth.lattice_mesh((5, 4, 3), L=1.0)  # 60 elements: 4 tiles, the last one ragged
    o, U = _state(mesh, k, nq)
    g = DG(mesh, k, nq1d=nq, mu=1e-2)
    g.set_tuning("fixed")
    w = torch.tensor(o.to_flat(U), device="cuda")
    v = torch.tensor(o.to_flat(np.random.default_rng(4).standard_normal(U.shape)), device="cuda")
    runs = {"fp64": (lambda: g.residual(w), lambda: g.jvp(w, v, shift=3.0)),
            "fp32": (lambda: g.residual(w, precision="fp32"), lambda: g.jvp(w, v, shift=3.0, mode="exact_fp32")),
            "bf16": (lambda: g.residual(w, precision="bf16"), lambda: g.jvp(w, v, shift=3.0, mode="exact_bf16"))}
    ref = {p: (f[0]().clone(), f[1]().clone()) for p, f in runs.items()}
    assert rel(ref["fp64"][1].cpu().numpy(), o.to_flat(o.operator(U, o.from_flat(v.cpu().numpy()), 3.0))) <= 1e-12
    n_run = 0
    for p, (res, jv) in runs.items():
        for jvp in (0, 1):
            for fused in (0, 1):
                for fo in (1, 2):
                    for vo in (1, 2):
                        try:
                            g.set_fine_shape(p, jvp, fo, vo, fused)
                        except DGError as e:
                            # only the FP64 P4 face kernel (its trace table fills the LDS) lacks occupancy 2
                            assert e.status == -1 and (k, p, fo) == (4, "fp64", 2), (p, jvp, fo, vo)
                            continue
                        out = (jv if jvp else res)()
                        assert torch.equal(out, ref[p][jvp]), (p, jvp, fused, fo, vo)
                        n_run += 1
            g.set_fine_shape(p, jvp, 0, 0, 0)
    assert n_run >= 40
    g.close()


def test_fused_gradients_at_full_size():
    """P4 24^3: the fused-gradient volume kernel (every occupancy) gives the
    bits of the two-kernel path, FP64 / FP32 / BF16, residual and Jv."""
    from paper_1809_00866_amd import DG
    from paper_1809_00866_amd._lib import DGError
    _say("fused gradients, P4 24^3")
    cfg, mesh, fld = synth.preset("cfg3")
    g = DG(mesh, cfg["order"], basis=cfg["space"], nq1d=cfg["nq1d"], flux="roe", mu=cfg["mu"])
    g.set_tuning("fixed")
    w = g.project_field(fld)
    v = torch.tensor(synth.random_vector(g.ndof, cfg["v_seed"]), device="cuda")
    modes = {"fp64": "exact", "fp32": "exact_fp32", "bf16": "exact_bf16"}
    for p, mode in modes.items():
        ref = (g.residual(w, precision=p).clone(), g.jvp(w, v, shift=2.0, mode=mode).clone())
        for jvp in (0, 1):
            for vo in (1, 2):
                try:
                    g.set_fine_shape(p, jvp, 0, vo, 1)
                except DGError:
                    continue
                out = g.jvp(w, v, shift=2.0, mode=mode) if jvp else g.residual(w, precision=p)
                assert torch.equal(out, ref[jvp]), (p, jvp, vo)
            g.set_fine_shape(p, jvp, 0, 0, 0)
    g.close()


@pytest.mark.parametrize("k,nq", [(2, 3), (3, 4)], ids=["P2-m50", "P3-m100"])
def test_every_block_apply_shape(k, nq):
    from paper_1809_00866_amd import DG
    from paper_1809_00866_amd._lib import DGError
    _say(f"block apply shapes P{k}")
    mesh = synth.lattice_mesh((3, 3, 2), L=1.0)
    o, U = _state(mesh, k, nq)
    g = DG(mesh, k, nq1d=nq, mu=1e-2)
    g.set_tuning("fixed")
    w = torch.tensor(o.to_flat(U), device="cuda")
    shift = 8.0
    R = np.random.default_rng(5).standard_normal(U.shape)
    r = torch.tensor(o.to_flat(R), device="cuda")
    z_o = o.to_flat(block_solve(o.block_diagonal(U, shift=shift), R.reshape(o.ne, -1)).reshape(U.shape))
    m = o.nvar * o.nb
    for storage, tol in (("fp64", 1e-12), ("fp32", 1e-6), ("bf16", 1e-5)):
        g.block_setup(w, shift, storage=storage)
        z_def = g.block_apply(r).cpu().numpy()
        if storage == "fp64":
            assert rel(z_def, z_o) <= 1e-12
        ok = 0
        for kind, t, e in APPLY_SHAPES:
            try:
                g.set_apply_shape(0, kind, t, e)
            except DGError as err:
                assert err.status == -1
                assert kind == "row" and m > 64 or kind == "vec" and t == 64 and m > 64, (storage, kind, t, e)
                continue
            z = g.block_apply(r).cpu().numpy()
            if storage == "fp64":
                assert rel(z, z_o) <= tol, (kind, t, e)
            else:
                assert rel(z, z_def) <= tol, (storage, kind, t, e)
            ok += 1
        assert ok >= 4
    g.close()


@pytest.fixture(scope="module")
def hierarchy():
    from paper_1809_00866_amd import DG
    _say("P3/P2/P1 hierarchy: oracle set-up")
    mesh = synth.lattice_mesh((3, 2, 2), L=1.0)
    o, U = _state(mesh, 3, 4, seed=21)
    shift, orders, iters = 6.0, (3, 2, 1), (2, 2, 6)
    mg = PMultigrid(o, U, shift, orders, iters)
    g = DG(mesh, 3, nq1d=4, mu=1e-2)
    g.set_tuning("fixed")
    w = torch.tensor(o.to_flat(U), device="cuda")
    yield dict(o=o, U=U, mg=mg, g=g, w=w, shift=shift, orders=orders, iters=iters)
    g.close()


def test_every_bsr_shape_matches_the_inherited_operators(hierarchy):
    from paper_1809_00866_amd._lib import DGError
    h = hierarchy
    o, mg, g = h["o"], h["mg"], h["g"]
    g.mg_setup(h["w"], h["shift"], h["orders"], h["iters"], storage="fp64", use_graph=True)
    rng = np.random.default_rng(7)
    R = rng.standard_normal(h["U"].shape)
    z_o = o.to_flat(mg.apply(R))
    r = torch.tensor(o.to_flat(R), device="cuda")
    for l in (1, 2):
        X = rng.standard_normal((o.ne, o.nvar, mg.nbs[l]))
        y_o = (mg.A[l] @ X.reshape(-1)).reshape(X.shape)
        x = torch.tensor(_flat(X), device="cuda")
        m = o.nvar * mg.nbs[l]
        ok = 0
        for bs, rpt, cs in BSR_SHAPES:
            try:
                g.set_bsr_shape(l, bs, rpt, cs)
            except DGError as err:
                assert err.status == -1 and not bsr_fits(bs, rpt, cs, m, 8), (l, bs, rpt, cs)
                continue
            assert bsr_fits(bs, rpt, cs, m, 8), (l, bs, rpt, cs)
            y = _unflat(g.mg_level_apply(l, x).cpu().numpy(), o.ne, o.nvar, mg.nbs[l])
            assert np.linalg.norm(y - y_o) <= 1e-12 * np.linalg.norm(y_o), (l, bs, rpt, cs)
            ok += 1
        assert ok >= 20
        g.set_bsr_shape(l, 512, 0, 4)
    _say("V-cycle with pinned coarse shapes")
    for (b1, b2, a1, a2) in [((512, 1, 8), (1024, 2, 1), ("vec", 64, 2), ("row", 64, 8)),
                             ((1024, 2, 2), (256, 1, 4), ("row", 64, 1), ("vec", 128, 1))]:
        g.set_bsr_shape(1, *b1)
        g.set_bsr_shape(2, *b2)
        g.set_apply_shape(1, *a1)
        g.set_apply_shape(2, *a2)
        z = g.mg_apply(r).cpu().numpy()
        assert rel(z, z_o) <= 1e-9


def test_every_bsr_shape_of_the_fp32_copies_in_the_cycle(hierarchy, storage="fp32", elem=4, to_oracle=1e-4):
    """With FP32 storage the cycle applies FP32 copies of the coarse operators
    (FP64 sums); every block-sparse shape of those copies gives the V-cycle of
    the built-in shape to 1e-5 relative (the same FP32 products, summed in
    another order, through a nonlinear cycle), and the default cycle stays
    within 1e-4 of the oracle's FP64 cycle."""
    from paper_1809_00866_amd._lib import DGError
    h = hierarchy
    o, mg, g = h["o"], h["mg"], h["g"]
    g.set_tuning("fixed")
    g.mg_setup(h["w"], h["shift"], h["orders"], h["iters"], storage=storage, use_graph=True)
    R = np.random.default_rng(11).standard_normal(h["U"].shape)
    r = torch.tensor(o.to_flat(R), device="cuda")
    z_def = g.mg_apply(r).cpu().numpy()
    assert rel(z_def, o.to_flat(mg.apply(R))) <= to_oracle
    assert f"({storage} blocks)" in g.tuning_report()
    for l in (1, 2):
        m = o.nvar * mg.nbs[l]
        ok = 0
        for bs, rpt, cs in BSR_SHAPES:
            try:
                g.set_bsr_shape(l, bs, rpt, cs)
            except DGError as err:
                assert err.status == -1 and not bsr_fits(bs, rpt, cs, m, elem), (l, bs, rpt, cs)
                continue
            assert bsr_fits(bs, rpt, cs, m, elem), (l, bs, rpt, cs)
            assert rel(g.mg_apply(r).cpu().numpy(), z_def) <= 1e-5, (l, bs, rpt, cs)
            ok += 1
        assert ok >= 25
        g.set_bsr_shape(l, 512, 0, 4)


def test_autotuned_setup_matches_the_fixed_one(hierarchy):
    h = hierarchy
    o, mg, g, w = h["o"], h["mg"], h["g"], h["w"]
    rng = np.random.default_rng(9)
    V = rng.standard_normal(h["U"].shape)
    v = torch.tensor(o.to_flat(V), device="cuda")
    r = torch.tensor(o.to_flat(rng.standard_normal(h["U"].shape)), device="cuda")
    g.set_tuning("fixed")
    g.mg_setup(w, h["shift"], h["orders"], h["iters"], storage="fp64", use_graph=True)
    rep_fixed = g.tuning_report()
    jv_f = g.jvp(w, v, shift=2.0).clone()
    za_f = g.block_apply(r).cpu().numpy()
    zc_f = g.mg_apply(r).cpu().numpy()
    _say("tuned set-up")
    g.set_tuning("auto")
    g.autotune(w)
    g.mg_setup(w, h["shift"], h["orders"], h["iters"], storage="fp64", use_graph=True)
    rep = g.tuning_report()
    _say(rep)
    assert torch.equal(g.jvp(w, v, shift=2.0), jv_f)
    assert rel(g.block_apply(r).cpu().numpy(), za_f) <= 1e-13
    assert rel(g.mg_apply(r).cpu().numpy(), zc_f) <= 1e-10
    assert "mode fixed" in rep_fixed and "(default)" in rep_fixed
    assert "mode auto" in rep and "(not tuned)" not in rep
    assert "mg level 1 (P2, m=50)" in rep and "mg level 2 (P1, m=20)" in rep
    # the tuned choices are cached: an eager cycle set up again equals the graph replay
    z_graph = g.mg_apply(r).cpu().numpy()
    g.mg_setup(w, h["shift"], h["orders"], h["iters"], storage="fp64", use_graph=False)
    assert g.tuning_report() == rep
    assert np.array_equal(g.mg_apply(r).cpu().numpy(), z_graph)
    g.set_tuning("fixed")
