"""dg_jvp_noalloc (exact Jv with the intermediate arrays in the library's static
device scratch) against dg_jvp (the same kernels with the context's own
buffers), through the C ABI.

Both calls run the same kernels on the same inputs, so the results must be
equal bit for bit (stronger than the 1e-12 FP64 parity bar); the smaller case
is also checked against the oracle at 1e-12.  Two calls in a row share the
scratch, the second on a smaller mesh; the affine MFMA path (3D P3), the
curved path and the 2D reference path are covered, and a context whose arrays
exceed the scratch is refused with DG_ERR_ARG before any launch.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import DGOracle, NavierStokes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(N, order, nq, perturb=0.0, seed=5):
    from paper_1809_00866_amd import DG
    mesh = synth.lattice_mesh(N, L=1.0, perturb=perturb, seed=seed if perturb else None)
    d = len(N)
    o = DGOracle(mesh, order, "P", nq, NavierStokes(d, mu=1e-2))
    fld = synth.TaylorGreenStandIn(seed=seed, L=1.0) if d == 3 else synth.FreeStreamPlusModes(seed=seed)
    U = o.project(fld)
    g = DG(mesh, order, nq1d=nq, mu=1e-2)
    w = torch.tensor(o.to_flat(U), device="cuda")
    V = np.random.default_rng(seed + 1).standard_normal(U.shape)
    v = torch.tensor(o.to_flat(V), device="cuda")
    return o, g, U, V, w, v


@pytest.mark.parametrize("kind", ["affine-P3", "curved-P2", "2d-P2"])
def test_noalloc_jvp_equals_dg_jvp_on_two_calls_the_second_smaller(kind):
    big, small = {
        "affine-P3": (((6, 5, 4), 3, 4, 0.0), ((2, 3, 2), 3, 4, 0.0)),
        "curved-P2": (((4, 3, 3), 2, 3, 0.1), ((2, 2, 2), 2, 3, 0.1)),
        "2d-P2": (((9, 7), 2, 4, 0.0), ((3, 2), 2, 4, 0.0)),
    }[kind]
    shift = 3.25
    results = []
    for N, k, nq, pert in (big, small):
        _say(f"noalloc {kind}: mesh {N}")
        o, g, U, V, w, v = _case(N, k, nq, pert)
        ref = g.jvp(w, v, shift=shift)
        out = g.jvp_noalloc(w, v, shift=shift)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (N, float((out - ref).abs().max()))
        results.append((o, U, V, out.cpu().numpy()))
        g.close()
    o, U, V, out = results[-1]
    J = o.to_flat(o.jvp(U, V) + shift * V)
    assert np.linalg.norm(out - J) <= 1e-12 * np.linalg.norm(J)


def test_noalloc_refuses_a_context_larger_than_the_scratch():
    from paper_1809_00866_amd import DG
    from paper_1809_00866_amd._lib import DGError
    _say("noalloc size limit")
    cap = DG.noalloc_scratch_bytes()
    assert cap == 256 << 20
    # P4 lattice: 11,400 bytes of scratch per element; 32 x 32 x 24 = 24,576 elements > 23,546
    g = DG(synth.lattice_mesh((32, 32, 24), L=1.0), 4, nq1d=5, mu=1e-2)
    w = torch.ones(g.ndof, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(w)
    out = torch.full_like(w, 7.0)
    with pytest.raises(DGError) as ei:
        g.jvp_noalloc(w, v, out=out)
    assert ei.value.status == -1
    assert torch.all(out == 7.0)          # nothing was launched
    g.close()
