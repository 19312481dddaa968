"""CPU tests of the C ABI: the library loads, exports every declared symbol,
and rejects invalid arguments on the host before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from paper_1809_00866_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTED) == names


def _create(prm, mesh):
    lib = L.load()
    xyz = np.ascontiguousarray(mesh["elem_xyz"], dtype=np.float64)
    nbr = np.ascontiguousarray(mesh["elem_nbr"], dtype=np.int64)
    m = L.DGMesh(xyz.shape[0], xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    h = ctypes.c_void_p()
    st = lib.dg_create(ctypes.byref(prm), ctypes.byref(m), ctypes.byref(h))
    return st, lib.dg_last_error().decode()


def _prm(dim=3, order=3, nq=4, basis=L.DG_BASIS_PK, flux=L.DG_FLUX_ROE):
    return L.DGParams(dim, order, basis, nq, flux, 1.4, 0.72, 1e-3, 0.0, 0.0)


@pytest.mark.parametrize("bad", [dict(dim=4), dict(order=-1), dict(nq=0), dict(basis=7), dict(flux=9)])
def test_create_rejects_bad_params(bad):
    kw = dict(dim=3, order=3, nq=4)
    kw.update(bad)
    st, msg = _create(_prm(**kw), synth.lattice_mesh((2, 2, 2)))
    assert st == -1 and msg


def test_create_accepts_curved_meshes_and_rejects_inverted_elements():
    """A perturbed lattice is a valid curved mesh (no argument error; without
    a GPU the create then fails on device memory); an element whose corners
    are mirrored has a negative Jacobian and is refused before device work."""
    st, msg = _create(_prm(), synth.lattice_mesh((2, 2, 2), perturb=0.1, seed=1))
    assert st != -1, msg
    mesh = synth.lattice_mesh((2, 2, 2), perturb=0.1, seed=1)
    xyz = np.array(mesh["elem_xyz"])
    xyz[3] = xyz[3][[1, 0, 3, 2, 5, 4, 7, 6]]            # mirror element 3 in x
    st, msg = _create(_prm(), dict(mesh, elem_xyz=xyz))
    assert st == -1 and "Jacobian" in msg


def test_create_rejects_nonconforming_curved_faces():
    """Rotating one element's local frame by 90 degrees about z keeps its
    Jacobian positive but makes its +-x faces disagree with the neighbour
    list: the face points seen from both sides no longer coincide."""
    mesh = synth.lattice_mesh((2, 2, 2), perturb=0.1, seed=1)
    xyz = np.array(mesh["elem_xyz"])
    old = xyz[3].copy()
    for i in range(2):
        for j in range(2):
            for k in range(2):
                xyz[3][i + 2 * j + 4 * k] = old[(1 - j) + 2 * i + 4 * k]
    st, msg = _create(_prm(), dict(mesh, elem_xyz=xyz))
    assert st == -1 and "not conforming" in msg


def test_create_rejects_inconsistent_neighbours():
    mesh = synth.lattice_mesh((3, 3, 3))
    mesh["elem_nbr"] = mesh["elem_nbr"].copy()
    mesh["elem_nbr"][4, 1] = 7
    st, msg = _create(_prm(), mesh)
    assert st == -1 and "neighbour" in msg


def test_create_rejects_uncompiled_configuration():
    st, msg = _create(_prm(order=6, nq=7), synth.lattice_mesh((2, 2, 2)))
    assert st == -1 and "no kernel compiled" in msg


def test_null_arguments():
    lib = L.load()
    assert lib.dg_create(None, None, None) == -1
    assert lib.dg_residual(None, None, None, None) == -1
    assert lib.dg_ndof(None) == -1
    assert lib.dg_mg_setup(None, None, 0.0, None, None) == -1
    assert lib.dg_mg_apply(None, None, None, None) == -1
    assert lib.dg_mg_level_apply(None, 0, None, None, None) == -1
    assert lib.dg_mg_update_fine(None, None, 0.0, 1, None) == -1
    assert lib.dg_rosenbrock_step(None, None, 0.1, None, None, None, None, None) == -1
    assert lib.dg_set_tuning(None, L.DG_TUNE_AUTO) == -1
    assert lib.dg_set_block_probing(None, L.DG_PROBE_AUTO) == -1
    assert lib.dg_autotune(None, None, None) == -1
    assert lib.dg_tuning_report(None, None, 0) == -1
    assert lib.dg_set_fine_shape(None, 0, 1, 1, 1, 0) == -1
    assert lib.dg_set_apply_shape(None, 0, 1, 64, 4) == -1
    assert lib.dg_set_bsr_shape(None, 1, 512, 2, 4) == -1


def test_create_checks_the_physics_model_on_the_host():
    """Unknown physics, the incompressible equations on a curved mesh and the
    Laplacian on a 3D curved mesh are refused before any device work."""
    prm = _prm(order=2, nq=3)
    prm.physics = 7
    st, msg = _create(prm, synth.lattice_mesh((2, 2, 2)))
    assert st == -1 and "physics" in msg
    prm.physics = L.DG_PHYS_INCOMPRESSIBLE
    st, msg = _create(prm, synth.lattice_mesh((2, 2, 2), perturb=0.1, seed=1))
    assert st == -1 and "lattice" in msg
    prm.physics = L.DG_PHYS_DIFFUSION  # the Laplacian on distorted meshes: 2D P2/P3/P6 only
    st, msg = _create(prm, synth.lattice_mesh((2, 2, 2), perturb=0.1, seed=1))
    assert st == -1 and "curved-element kernel" in msg
