"""Thin torch wrapper over the C ABI: device tensors in, device tensors out.

Every numerical step runs in libdg.so; this module only checks tensor
shapes/dtypes/devices and passes raw pointers plus the current HIP stream.
"""
import ctypes
import math

import numpy as np
import torch

from . import _lib as L

_FLUX = {"lf": L.DG_FLUX_LF, "roe": L.DG_FLUX_ROE}
_BASIS = {"P": L.DG_BASIS_PK, "Q": L.DG_BASIS_QK}
_MODE = {"exact": L.DG_JVP_EXACT, "fd": L.DG_JVP_FD, "exact_fp32": L.DG_JVP_EXACT_FP32, "stab": L.DG_JVP_STAB,
         "exact_bf16": L.DG_JVP_EXACT_BF16}
_STORAGE = {"fp64": L.DG_FP64, "fp32": L.DG_FP32, "bf16": L.DG_BF16}
_PREC = {"none": L.DG_PREC_NONE, "bj": L.DG_PREC_BJ, "mg": L.DG_PREC_MG, "mlp": L.DG_PREC_MLP}
_ORTH = {"cgs2": L.DG_ORTH_CGS2, "mgs": L.DG_ORTH_MGS}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _nb(k, d):
    return math.comb(k + d, d)


class DG:
    """A DG discretisation on a periodic lattice (see include/dg.h)."""

    def __init__(self, mesh, order, basis="P", nq1d=None, flux="roe", gamma=1.4, prandtl=0.72, mu=1e-3,
                 eta=0.0, entropy_fix=0.0, physics="compressible", beta=1.0, device="cuda"):
        """physics "compressible" (conserved rho, rho u, rho E), "incompressible"
        (u, p; mu is the kinematic viscosity, beta the artificial compressibility
        speed of the interface flux) or "diffusion" (scalar BR2 Laplacian, mu
        the diffusivity)."""
        self.lib = L.load()
        self.dim = int(mesh["dim"])
        self.order = int(order)
        self.nq1d = int(nq1d if nq1d is not None else order + 1)
        self.device = torch.device(device)
        phys = {"compressible": L.DG_PHYS_COMPRESSIBLE, "incompressible": L.DG_PHYS_INCOMPRESSIBLE,
                "diffusion": L.DG_PHYS_DIFFUSION}[physics]
        prm = L.DGParams(self.dim, self.order, _BASIS[basis], self.nq1d, _FLUX[flux], gamma, prandtl, mu, eta,
                         entropy_fix, phys, beta)
        xyz = np.ascontiguousarray(mesh["elem_xyz"], dtype=np.float64)
        nbr = np.ascontiguousarray(mesh["elem_nbr"], dtype=np.int64)
        m = L.DGMesh(xyz.shape[0], xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.dg_create(ctypes.byref(prm), ctypes.byref(m), ctypes.byref(h)), "dg_create")
        self.ctx = h
        self.ne = xyz.shape[0]
        self.ndof = self.lib.dg_ndof(h)
        self.nb = self.lib.dg_nbasis(h)
        self.nv = self.lib.dg_nvar(h)
        self.nq = self.lib.dg_nq(h)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.dg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- helpers
    def _vec(self, t, name):
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
                and t.numel() == self.ndof):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor with {self.ndof} entries")
        return t

    def empty(self):
        return torch.empty(self.ndof, dtype=torch.float64, device=self.device)

    # ---------------------------------------------------------------- entry points
    def volume_points(self):
        xyz = torch.empty((self.dim, self.nq, self.ne), dtype=torch.float64, device=self.device)
        L.check(self.lib.dg_volume_points(self.ctx, _ptr(xyz), _stream()), "dg_volume_points")
        return xyz

    def project(self, f):
        """f: [nvar][nq][n_elem] values at the volume points -> DOF vector."""
        f = f.contiguous()
        if f.shape != (self.nv, self.nq, self.ne) or f.dtype != torch.float64 or not f.is_cuda:
            raise ValueError("f must be float64 CUDA [nvar, nq, n_elem]")
        w = self.empty()
        L.check(self.lib.dg_project(self.ctx, _ptr(f), _ptr(w), _stream()), "dg_project")
        return w

    def project_field(self, field):
        """Evaluate a host field function at the volume points and project on the GPU."""
        xyz = self.volume_points().cpu().numpy()            # [dim, nq, ne]
        vals = field(np.moveaxis(xyz, 0, -1))                # [nq, ne, nvar]
        f = torch.from_numpy(np.ascontiguousarray(np.moveaxis(vals, -1, 0))).to(self.device)
        return self.project(f)

    def residual(self, w, out=None, precision="fp64"):
        self._vec(w, "w")
        out = self.empty() if out is None else self._vec(out, "out")
        if precision == "fp32":
            L.check(self.lib.dg_residual_fp32(self.ctx, _ptr(w), _ptr(out), _stream()), "dg_residual_fp32")
        elif precision == "bf16":
            L.check(self.lib.dg_residual_bf16(self.ctx, _ptr(w), _ptr(out), _stream()), "dg_residual_bf16")
        else:
            L.check(self.lib.dg_residual(self.ctx, _ptr(w), _ptr(out), _stream()), "dg_residual")
        return out

    def jvp(self, w, v, shift=0.0, mode="exact", r_w=None, out=None):
        self._vec(w, "w")
        self._vec(v, "v")
        if r_w is not None:
            self._vec(r_w, "r_w")
        out = self.empty() if out is None else self._vec(out, "out")
        L.check(self.lib.dg_jvp(self.ctx, _ptr(w), _ptr(r_w), _ptr(v), float(shift), _MODE[mode], _ptr(out),
                                _stream()), "dg_jvp")
        return out

    @staticmethod
    def noalloc_scratch_bytes():
        """Size of the static device scratch that dg_jvp_noalloc uses."""
        return int(L.load().dg_jvp_noalloc_scratch_bytes())

    def jvp_noalloc(self, w, v, shift=0.0, out=None):
        """shift*v + J(w) v through dg_jvp_noalloc (exact mode, static scratch)."""
        self._vec(w, "w")
        self._vec(v, "v")
        out = self.empty() if out is None else self._vec(out, "out")
        L.check(self.lib.dg_jvp_noalloc(self.ctx, _ptr(w), _ptr(v), float(shift), _ptr(out), _stream()),
                "dg_jvp_noalloc")
        return out

    def set_tuning(self, mode):
        """"auto" (time candidate launch shapes at setup, the default) or "fixed"
        (the built-in shapes, no timing)."""
        m = {"fixed": L.DG_TUNE_FIXED, "auto": L.DG_TUNE_AUTO}[mode]
        L.check(self.lib.dg_set_tuning(self.ctx, m), "dg_set_tuning")

    def set_block_probing(self, mode):
        """"auto" (element-local probing of the diagonal blocks where the kernels
        allow it, the default) or "coloured" (one Jv per column and colour)."""
        m = {"auto": L.DG_PROBE_AUTO, "coloured": L.DG_PROBE_COLOURED}[mode]
        L.check(self.lib.dg_set_block_probing(self.ctx, m), "dg_set_block_probing")

    def autotune(self, w):
        """Time and select the fine operator's launch shapes at state w (and the
        block apply shape when block factors exist)."""
        self._vec(w, "w")
        L.check(self.lib.dg_autotune(self.ctx, _ptr(w), _stream()), "dg_autotune")

    def tuning_report(self):
        """The context's launch shapes, one line per kernel family."""
        buf = ctypes.create_string_buffer(8192)
        L.check(self.lib.dg_tuning_report(self.ctx, buf, len(buf)), "dg_tuning_report")
        return buf.value.decode()

    def set_fine_shape(self, precision, jvp, face_occ, volume_occ, fused_gradients=False):
        """Pin the waves per SIMD (1, 2; 0 = default) of the MFMA face and volume
        kernels of the operator of `precision`, residual (jvp False) or Jv, and
        whether the volume kernel forms the corrected gradients itself."""
        L.check(self.lib.dg_set_fine_shape(self.ctx, _STORAGE[precision], int(bool(jvp)), int(face_occ),
                                           int(volume_occ), int(bool(fused_gradients))), "dg_set_fine_shape")

    def set_apply_shape(self, level, kind, threads=0, epw=0):
        """Pin the block-inverse apply shape of level 0 (fine block Jacobi) or a
        coarse level: kind "default", "row" (threads 64) or "vec"."""
        k = {"default": 0, "row": 1, "vec": 2}[kind]
        L.check(self.lib.dg_set_apply_shape(self.ctx, int(level), k, int(threads), int(epw)), "dg_set_apply_shape")

    def set_bsr_shape(self, level, workgroup, rows_per_thread, column_slices):
        """Pin coarse level `level`'s block-sparse apply shape."""
        L.check(self.lib.dg_set_bsr_shape(self.ctx, int(level), int(workgroup), int(rows_per_thread),
                                          int(column_slices)), "dg_set_bsr_shape")

    def block_setup(self, w, shift, storage="fp64"):
        self._vec(w, "w")
        L.check(self.lib.dg_block_precond_setup(self.ctx, _ptr(w), float(shift), _STORAGE[storage], _stream()),
                "dg_block_precond_setup")

    def block_apply(self, r, out=None):
        self._vec(r, "r")
        out = self.empty() if out is None else self._vec(out, "out")
        L.check(self.lib.dg_block_precond_apply(self.ctx, _ptr(r), _ptr(out), _stream()), "dg_block_precond_apply")
        return out

    def mg_setup(self, w, shift, orders, smooth_iters, storage="fp64", use_graph=True, fine_precision="fp64",
                 cycle="v", rescale=False, coarse_ilu=False):
        """p-multigrid hierarchy at (w, shift); orders[0] must be the context's order;
        cycle "v" (Alg. vcic) or "full" (Alg. fullvcic)."""
        if cycle not in ("v", "full"):
            raise ValueError("cycle must be 'v' or 'full'")
        self._vec(w, "w")
        orders, smooth_iters = list(orders), list(smooth_iters)
        if not (2 <= len(orders) <= 3) or len(smooth_iters) != len(orders):
            raise ValueError("need 2 or 3 levels and one smoothing count per level")
        o = L.MgOpts(len(orders), (ctypes.c_int * 3)(*(orders + [0] * (3 - len(orders)))),
                     (ctypes.c_int * 3)(*(smooth_iters + [0] * (3 - len(orders)))), _STORAGE[storage],
                     int(bool(use_graph)), _STORAGE[fine_precision], L.DG_MG_FULL if cycle == "full" else L.DG_MG_V,
                     int(bool(rescale)), int(bool(coarse_ilu)))
        self.mg_levels = [(self.ne * self.nv * _nb(k, self.dim)) for k in orders]
        L.check(self.lib.dg_mg_setup(self.ctx, _ptr(w), float(shift), ctypes.byref(o), _stream()), "dg_mg_setup")

    def mg_update_fine(self, w, shift, refresh_blocks=True):
        """Lag the hierarchy: the fine-level operator follows (w, shift), the coarse
        operators stay those of the last mg_setup."""
        self._vec(w, "w")
        L.check(self.lib.dg_mg_update_fine(self.ctx, _ptr(w), float(shift), int(bool(refresh_blocks)), _stream()),
                "dg_mg_update_fine")

    def mg_apply(self, r, out=None):
        self._vec(r, "r")
        out = self.empty() if out is None else self._vec(out, "out")
        L.check(self.lib.dg_mg_apply(self.ctx, _ptr(r), _ptr(out), _stream()), "dg_mg_apply")
        return out

    def mg_level_apply(self, level, x):
        n = self.mg_levels[level]
        if not (isinstance(x, torch.Tensor) and x.dtype == torch.float64 and x.is_cuda and x.is_contiguous()
                and x.numel() == n):
            raise ValueError(f"x must be a contiguous float64 CUDA tensor with {n} entries")
        y = torch.empty_like(x)
        L.check(self.lib.dg_mg_level_apply(self.ctx, int(level), _ptr(x), _ptr(y), _stream()), "dg_mg_level_apply")
        return y

    # ---------------------------------------------------------------- learned preconditioner
    def _f32(self, t, name, n):
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float32 and t.is_cuda and t.is_contiguous()
                and t.numel() == n):
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor with {n} entries")
        return t

    @property
    def mlp_sizes(self):
        n_out = self.nv * self.nb
        return n_out + 2 * self.dim * self.nv, n_out

    def mlp_nparams(self):
        return int(self.lib.dg_mlp_nparams(self.ctx))

    def mlp_set_mode(self, mode):
        """"direct" (z = s MLP(x)) or "correct_bj" (z = D^-1 r + s MLP(x))."""
        m = {"direct": L.DG_MLP_DIRECT, "correct_bj": L.DG_MLP_CORRECT_BJ}[mode]
        L.check(self.lib.dg_mlp_set_mode(self.ctx, m), "dg_mlp_set_mode")

    def mlp_set_weights(self, theta):
        theta = torch.as_tensor(theta, dtype=torch.float32).to(self.device).contiguous()
        self._f32(theta, "theta", self.mlp_nparams())
        L.check(self.lib.dg_mlp_set_weights(self.ctx, _ptr(theta), _stream()), "dg_mlp_set_weights")

    def mlp_get_weights(self):
        out = torch.empty(self.mlp_nparams(), dtype=torch.float32, device=self.device)
        L.check(self.lib.dg_mlp_get_weights(self.ctx, _ptr(out), _stream()), "dg_mlp_get_weights")
        return out

    def mlp_features(self, w, r, z=None):
        """(X [ne, n_in], T [ne, n_out] or None, s [ne]) for state w, residual r, optional target z."""
        self._vec(w, "w")
        self._vec(r, "r")
        n_in, n_out = self.mlp_sizes
        X = torch.empty((self.ne, n_in), dtype=torch.float32, device=self.device)
        T = None if z is None else torch.empty((self.ne, n_out), dtype=torch.float32, device=self.device)
        s = torch.empty(self.ne, dtype=torch.float64, device=self.device)
        if z is not None:
            self._vec(z, "z")
        L.check(self.lib.dg_mlp_features(self.ctx, _ptr(w), _ptr(r), _ptr(z), _ptr(X), _ptr(T), _ptr(s), _stream()),
                "dg_mlp_features")
        return X, T, s

    def mlp_forward(self, X):
        n_in, n_out = self.mlp_sizes
        X = X.contiguous()
        self._f32(X, "X", X.shape[0] * n_in)
        Y = torch.empty((X.shape[0], n_out), dtype=torch.float32, device=self.device)
        L.check(self.lib.dg_mlp_forward(self.ctx, _ptr(X), X.shape[0], _ptr(Y), _stream()), "dg_mlp_forward")
        return Y

    def _batch(self, X, T, rows):
        n_in, n_out = self.mlp_sizes
        self._f32(X, "X", X.shape[0] * n_in)
        self._f32(T, "T", X.shape[0] * n_out)
        if rows is not None and not (rows.dtype == torch.int64 and rows.is_cuda and rows.is_contiguous()):
            raise ValueError("rows must be a contiguous int64 CUDA tensor")
        return rows.numel() if rows is not None else X.shape[0]

    def mlp_grad(self, X, T, rows=None):
        B = self._batch(X, T, rows)
        g = torch.empty(self.mlp_nparams(), dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        L.check(self.lib.dg_mlp_grad(self.ctx, _ptr(X), _ptr(T), _ptr(rows), B, _ptr(g), _ptr(loss), _stream()),
                "dg_mlp_grad")
        return g, loss

    def mlp_train_step(self, X, T, rows=None, lr=1e-3, loss=None):
        B = self._batch(X, T, rows)
        L.check(self.lib.dg_mlp_train_step(self.ctx, _ptr(X), _ptr(T), _ptr(rows), B, float(lr), _ptr(loss),
                                           _stream()), "dg_mlp_train_step")

    def mlp_apply(self, w, r, out=None):
        self._vec(w, "w")
        self._vec(r, "r")
        out = self.empty() if out is None else self._vec(out, "out")
        L.check(self.lib.dg_mlp_apply(self.ctx, _ptr(w), _ptr(r), _ptr(out), _stream()), "dg_mlp_apply")
        return out

    def fgmres(self, w, shift, b, x=None, restart=30, max_iter=1000, rtol=1e-8, precond="bj", jvp_mode="exact",
               rho_ref=0.0, judge_after=5, orth="cgs2", check_every=1):
        self._vec(w, "w")
        self._vec(b, "b")
        x = torch.zeros_like(b) if x is None else self._vec(x, "x")
        opts = L.SolveOpts(restart, max_iter, rtol, _PREC[precond], _MODE[jvp_mode], float(rho_ref), int(judge_after),
                           _ORTH[orth], int(check_every))
        st = L.SolveStats()
        status = self.lib.dg_fgmres_solve(self.ctx, _ptr(w), float(shift), _ptr(b), _ptr(x), ctypes.byref(opts),
                                          ctypes.byref(st), _stream())
        L.check(status, "dg_fgmres_solve", allow_not_converged=True)
        stats = {k: getattr(st, k) for k, _ in L.SolveStats._fields_}
        return x, stats

    def rosenbrock_step(self, w, dt, coeffs, out=None, restart=30, max_iter=1000, rtol=1e-8, precond="bj",
                        jvp_mode="exact"):
        """One step of Alg. ros; coeffs = dict(gamma, a, c, m) (a, c: n_s x n_s, m: n_s).
        The preconditioner must be set up at (w, 1/(gamma dt))."""
        self._vec(w, "w")
        out = self.empty() if out is None else self._vec(out, "out")
        ns = len(coeffs["m"])
        if not 1 <= ns <= L.ROS_MAX_STAGES:
            raise ValueError("1..6 stages")
        k = L.RosCoeffs()
        k.n_stages, k.gamma = ns, float(coeffs["gamma"])
        for s in range(ns):
            k.m[s] = float(coeffs["m"][s])
            for o in range(s):
                k.a[s][o] = float(coeffs["a"][s][o])
                k.c[s][o] = float(coeffs["c"][s][o])
        opts = L.SolveOpts(restart, max_iter, rtol, _PREC[precond], _MODE[jvp_mode], 0.0, 0, L.DG_ORTH_CGS2, 1)
        st = L.SolveStats()
        status = self.lib.dg_rosenbrock_step(self.ctx, _ptr(w), float(dt), ctypes.byref(k), ctypes.byref(opts),
                                             _ptr(out), ctypes.byref(st), _stream())
        L.check(status, "dg_rosenbrock_step", allow_not_converged=True)
        return out, {f: getattr(st, f) for f, _ in L.SolveStats._fields_}

    def max_wave_speed(self, w):
        self._vec(w, "w")
        out = ctypes.c_double()
        L.check(self.lib.dg_max_wave_speed(self.ctx, _ptr(w), ctypes.byref(out), _stream()), "dg_max_wave_speed")
        return out.value

    def set_profiling(self, on=True):
        L.check(self.lib.dg_set_profiling(self.ctx, int(bool(on))), "dg_set_profiling")

    def kernel_time(self, name):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        L.check(self.lib.dg_kernel_time(self.ctx, name.encode(), ctypes.byref(ms), ctypes.byref(n)),
                "dg_kernel_time")
        return ms.value, n.value

    def sync(self):
        L.check(self.lib.dg_sync(self.ctx), "dg_sync")
