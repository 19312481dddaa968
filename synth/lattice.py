"""Periodic structured lattices (no discretisation arithmetic).

Element numbering: e = i + Nx*(j + Ny*k).  Local vertices are lexicographic,
v = v0 + 2*v1 + 4*v2 with v_i in {0, 1} meaning the low / high end of the
element along axis i.  Local faces are ordered (-x, +x, -y, +y, -z, +z).

Vertex coordinates are stored per element and are *unwrapped*: the element at
the high end of a periodic axis spans [L - h, L], not [L - h, 0].  A seeded
perturbation moves every lattice vertex once, so the periodic images of a
vertex move together and faces stay conforming.
"""
import numpy as np


def _as_tuple(v, d):
    if np.isscalar(v):
        return (v,) * d
    v = tuple(v)
    assert len(v) == d
    return v


def mesh_neighbors(N):
    """Face-neighbour table [n_elem, 2*d] of a periodic lattice with N = (Nx, Ny[, Nz])."""
    N = tuple(int(n) for n in N)
    d = len(N)
    ne = int(np.prod(N))
    idx = np.arange(ne).reshape(N[::-1])  # idx[k, j, i] = e
    nbr = np.empty((ne, 2 * d), dtype=np.int64)
    for p in range(d):
        ax = d - 1 - p  # numpy axis of coordinate p
        nbr[:, 2 * p] = np.roll(idx, 1, axis=ax).reshape(-1)       # element at i-1
        nbr[:, 2 * p + 1] = np.roll(idx, -1, axis=ax).reshape(-1)  # element at i+1
    return nbr


def lattice_mesh(N, L=1.0, perturb=0.0, seed=None, origin=0.0):
    """Periodic lattice of N[0] x ... x N[d-1] elements on [origin, origin+L]^d.

    Returns a dict with
      elem_xyz : float64 [n_elem, 2^d, d]   unwrapped corner coordinates
      elem_nbr : int64   [n_elem, 2*d]      face neighbours (-x,+x,-y,+y,-z,+z)
      period   : float64 [d]                box lengths
      N, L, h  : lattice sizes
    perturb is the half-width of the uniform vertex noise as a fraction of h.
    """
    N = tuple(int(n) for n in N)
    d = len(N)
    L = np.array(_as_tuple(L, d), dtype=np.float64)
    h = L / np.array(N, dtype=np.float64)
    org = np.array(_as_tuple(origin, d), dtype=np.float64)
    ne = int(np.prod(N))

    # one perturbation per periodic lattice vertex
    if perturb != 0.0:
        rng = np.random.default_rng(seed)
        delta = rng.uniform(-1.0, 1.0, size=tuple(N[::-1]) + (d,)) * (perturb * h)
    else:
        delta = np.zeros(tuple(N[::-1]) + (d,))

    grids = np.meshgrid(*[np.arange(n) for n in N[::-1]], indexing="ij")
    ijk = [g.reshape(-1) for g in grids[::-1]]  # ijk[p][e]
    nv = 2 ** d
    xyz = np.empty((ne, nv, d), dtype=np.float64)
    for v in range(nv):
        bits = [(v >> p) & 1 for p in range(d)]
        lat = [ijk[p] + bits[p] for p in range(d)]
        wrapped = tuple(lat[p] % N[p] for p in range(d))[::-1]
        dv = delta[wrapped]
        for p in range(d):
            xyz[:, v, p] = org[p] + lat[p] * h[p] + dv[:, p]
    return {
        "elem_xyz": xyz,
        "elem_nbr": mesh_neighbors(N),
        "period": L.copy(),
        "N": N,
        "L": L,
        "h": h,
        "dim": d,
    }
