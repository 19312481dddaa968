"""Instrumented operation count of the pointwise steps of the residual and Jv.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The oracle's pointwise physics (volume flux F^c - F^v of the corrected
gradient, and at a face point the numerical flux H^c minus the viscous flux
of the averaged state and averaged corrected gradient, normal component) is
evaluated at one point on a counting number type instead of floats.  Each
value carries an optional tangent, so one evaluation counts either the
residual's pointwise work (values only) or the Jacobian-vector product's
(value and directional derivative, forward mode).  Costs per operation:

  operation        value only   value + tangent
  a + b, a - b         1          2  (1 if one operand has no tangent)
  a * b                1          4  (2 if one operand has no tangent)
  a / b                1          4  (2 if the divisor has no tangent)
  sqrt(a)              1          3
  -a, |a|, max         0          0  (sign changes and selections)

Additions of an exact 0 and products with an exact +-1 are free (numpy's
reductions start from 0).  These are the flops of the method's pointwise
formulas as the oracle writes them; the GPU kernels compute the same
quantities (rearranged), so the count is the algorithmic pointwise work
behind the roofline figures, next to the contraction count of the basis
products.
"""
import numpy as np

from .physics import NavierStokes


class Tally:
    flops = 0


def _val(x):
    return x.v if isinstance(x, Num) else float(x)


def _tan(x):
    return x.t if isinstance(x, Num) else None


def _free_const(x, k):
    return not isinstance(x, Num) and float(x) == k


class Num:
    """A float (and optionally its tangent) that counts its arithmetic."""
    __slots__ = ("v", "t")

    def __init__(self, v, t=None):
        self.v = float(v)
        self.t = None if t is None else float(t)

    # ---- arithmetic
    def _add(self, o, sign):
        if isinstance(o, np.ndarray):
            return NotImplemented
        if _free_const(o, 0.0):
            return self
        ot = _tan(o)
        Tally.flops += 2 if (self.t is not None and ot is not None) else 1
        t = None
        if self.t is not None or ot is not None:
            t = (self.t or 0.0) + sign * (ot or 0.0)
        return Num(self.v + sign * _val(o), t)

    def __add__(self, o):
        return self._add(o, 1.0)

    def __radd__(self, o):
        return self._add(o, 1.0)

    def __sub__(self, o):
        return self._add(o, -1.0)

    def __rsub__(self, o):
        if isinstance(o, np.ndarray):
            return NotImplemented
        return (-self)._add(o, 1.0)

    def __neg__(self):
        return Num(-self.v, None if self.t is None else -self.t)

    def __mul__(self, o):
        if isinstance(o, np.ndarray):
            return NotImplemented
        if _free_const(o, 1.0):
            return self
        if _free_const(o, -1.0):
            return -self
        ov, ot = _val(o), _tan(o)
        if self.t is None and ot is None:
            Tally.flops += 1
            return Num(self.v * ov)
        if self.t is not None and ot is not None:
            Tally.flops += 4
            return Num(self.v * ov, self.t * ov + self.v * ot)
        Tally.flops += 2
        return Num(self.v * ov, (self.t if self.t is not None else 0.0) * ov + (self.v * ot if ot is not None else 0.0))

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, np.ndarray):
            return NotImplemented
        ov, ot = _val(o), _tan(o)
        q = self.v / ov
        if self.t is None and ot is None:
            Tally.flops += 1
            return Num(q)
        if ot is None:
            Tally.flops += 2
            return Num(q, self.t / ov)
        Tally.flops += 4
        return Num(q, ((self.t or 0.0) - q * ot) / ov)

    def __rtruediv__(self, o):
        if isinstance(o, np.ndarray):
            return NotImplemented
        return Num(o) / self

    def sqrt(self):
        s = np.sqrt(self.v)
        if self.t is None:
            Tally.flops += 1
            return Num(s)
        Tally.flops += 3
        return Num(s, self.t / (2.0 * s))

    # ---- selections (branches decided on the value)
    def __ge__(self, o):
        return self.v >= _val(o)

    def __gt__(self, o):
        return self.v > _val(o)

    def __le__(self, o):
        return self.v <= _val(o)

    def __lt__(self, o):
        return self.v < _val(o)

    @property
    def real(self):
        return self


def _nums(vals, tans):
    """Object array of Num with a leading batch axis of length 1 (the oracle's
    physics works on batches of points)."""
    vals = np.asarray(vals, dtype=np.float64)[None]
    tans = None if tans is None else np.asarray(tans, dtype=np.float64)[None]
    out = np.empty(vals.shape, dtype=object)
    for idx in np.ndindex(out.shape):
        out[idx] = Num(vals[idx], None if tans is None else tans[idx])
    return out


def _count(fn):
    Tally.flops = 0
    fn()
    return Tally.flops


def pointwise_flops(dim=3, flux="roe", gamma=1.4, prandtl=0.72, mu=1e-3, seed=0):
    """Flops of the pointwise steps at one point, as a dict:
      vol_res, vol_jvp: volume flux F = F^c(u) - F^v(u, G) (G = grad u + R,
        the sum counted here) without / with the tangent;
      face_res, face_jvp: face flux H^c(uL, uR, n) - F^v({u}, {grad u} +
        eta {r}) . n, with the averages formed at the point.
    The state is a generic smooth one (no branch depends on it in a way that
    changes the count except the entropy-fix switch of the Roe flux, which is
    inactive here: the larger count)."""
    ns = NavierStokes(dim, gamma=gamma, prandtl=prandtl, mu=mu, flux=flux)
    n = dim + 2
    rng = np.random.default_rng(seed)
    u0 = np.concatenate([[1.0], 0.3 * rng.standard_normal(dim), [2.5 + 0.1 * rng.standard_normal()]])
    G0 = 0.1 * rng.standard_normal((n, dim))
    R0 = 0.01 * rng.standard_normal((n, dim))
    du, dG, dR = (rng.standard_normal(s) for s in ((n,), (n, dim), (n, dim)))
    nrm = rng.standard_normal(dim)
    nrm /= np.linalg.norm(nrm)
    out = {}
    for tag, jvp in (("res", False), ("jvp", True)):
        def vol():
            u = _nums(u0, du if jvp else None)
            G = _nums(G0, dG if jvp else None) + _nums(R0, dR if jvp else None)
            ns.conv_flux(u) - ns.visc_flux(u, G)

        def face():
            uL = _nums(u0, du if jvp else None)
            uR = _nums(u0 * (1 + 0.01 * np.arange(n)), du[::-1].copy() if jvp else None)
            gL = _nums(G0, dG if jvp else None)
            gR = _nums(G0[::-1].copy(), dG[::-1].copy() if jvp else None)
            rL = _nums(R0, dR if jvp else None)
            rR = _nums(-R0, -dR if jvp else None)
            gface = 0.5 * (gL + gR) + ns.eta * 0.5 * (rL + rR)
            uavg = 0.5 * (uL + uR)
            Fv = ns.visc_flux(uavg, gface)
            ns.conv_numflux(uL, uR, nrm[None]) - np.einsum("...pc,...p->...c", Fv, nrm[None])

        out["vol_" + tag] = _count(vol)
        out["face_" + tag] = _count(face)
        if flux == "roe":
            # np.where evaluates both operands of the entropy-fix switch; the
            # fixed value (lam^2 + delta^2)/(2 delta) is not taken on any of
            # the three waves here, so its cost is taken out again
            lam, delta = Num(0.3, 0.1 if jvp else None), Num(0.2, 0.2 if jvp else None)
            out["face_" + tag] -= 3 * _count(lambda: (lam * lam + delta * delta) / (2.0 * delta))
    return out
