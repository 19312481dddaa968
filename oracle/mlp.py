"""Learned element-local preconditioner -- FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The flexible outer solver (Sec. 2.5) accepts a preconditioner that changes
from one application to the next, so a trained network may stand in for
(or alternate with) element-wise block Jacobi.  Definition used here (the
paper does not specify one; the choices are listed with the other readings):

* features of element K: the element's residual slice r_K (n*Nb values, local
  order c*Nb + b) divided by s_K = ||r_K||_2 + 1e-300, then for every face
  neighbour f (order -x,+x,-y,+y,-z,+z) the cell means of the n conserved
  variables of the linearisation state divided by their RMS over the mesh;
* a multilayer perceptron n_in -> 256 -> 256 -> n*Nb with ReLU after the two
  hidden layers, trained and applied in BF16 mixed precision: every operand
  of every matrix product is a BF16 number (round to nearest even) -- in the
  forward pass the inputs, weights and hidden activations, in the backward
  pass also the output gradient and the back-propagated deltas -- while
  sums, biases, the ReLU masks and the master weights keep full precision
  (FP32 on the device, FP64 here).  round_deltas=False gives the narrower
  reading that rounds only the forward operands;
* output z_K = s_K * MLP(x_K) (positively homogeneous in r), or in the
  block-Jacobi correction mode z_K = D_K^{-1} r_K + s_K * MLP(x_K), where a
  network with a zero last layer is block Jacobi exactly;
* training: mean squared error on the normalised targets t_K = z_K / s_K
  (correction mode: (z_K - D_K^{-1} r_K) / s_K), Adam (beta1 0.9, beta2
  0.999, eps 1e-8), FP32 master weights.

Parameter vector (flat, FP32 on the device): W1 [256 x n_in], b1 [256],
W2 [256 x 256], b2 [256], W3 [n_out x 256], b3 [n_out] (row-major, rows =
outputs).
"""
import numpy as np

HIDDEN = 256


def bf16_round(x):
    """Round to the nearest BF16 value, ties to even (8-bit significand)."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    finite = np.isfinite(a)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    r = np.where(finite, r, u & 0xFFFF0000)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def sizes(nvar, nb, nfaces):
    n_out = nvar * nb
    return nvar * nb + nfaces * nvar, HIDDEN, n_out


def split(theta, n_in, n_out):
    """Views W1, b1, W2, b2, W3, b3 of the flat parameter vector."""
    shapes = [(HIDDEN, n_in), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (n_out, HIDDEN), (n_out,)]
    out, k = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(theta[k:k + n].reshape(s))
        k += n
    assert k == theta.size
    return out


def n_params(n_in, n_out):
    return HIDDEN * n_in + HIDDEN + HIDDEN * HIDDEN + HIDDEN + n_out * HIDDEN + n_out


def cell_means(o, U):
    """Cell means (1/|K|) int_K u_c of every element, [ne, nvar], by quadrature."""
    et = o.elem_tables(np.arange(o.ne))
    vals = np.einsum("eqb,ecb->eqc", et["phi"], U)
    return np.einsum("eq,eqc->ec", et["wdet"], vals) / et["wdet"].sum(axis=1)[:, None]


def block_apply(D, R):
    """D_K^{-1} r_K for blocks D[e, m, m] and R[e, c, b] (LU solve), as [e, c, b]."""
    ne = R.shape[0]
    return np.linalg.solve(D, R.reshape(ne, -1)[..., None])[..., 0].reshape(R.shape)


def targets(R, Z, D=None):
    """Normalised targets z_K / s_K, or (z_K - D_K^{-1} r_K) / s_K when the
    blocks D are given (correction mode), as [ne, n*Nb]."""
    ne = R.shape[0]
    s = np.linalg.norm(R.reshape(ne, -1), axis=1) + 1e-300
    Y = Z if D is None else Z - block_apply(D, R)
    return Y.reshape(ne, -1) / s[:, None]


def features(o, U, R):
    """Network inputs X [ne, n_in] and scales s [ne] for residual R[e, c, b] at state U."""
    r = R.reshape(o.ne, -1)
    s = np.linalg.norm(r, axis=1) + 1e-300
    mean = cell_means(o, U)
    mref = np.sqrt(np.mean(mean ** 2, axis=0)) + 1e-300
    nb = (mean / mref)[o.nbr]                        # [ne, nfaces, nvar]
    return np.concatenate([r / s[:, None], nb.reshape(o.ne, -1)], axis=1), s


def forward(theta, X, n_out, rounding=True):
    """Y = MLP(X) for a batch X [B, n_in]; returns Y and the activations.
    rounding: BF16 inputs, weights and hidden activations (the device's
    storage); False gives the plain FP64 network."""
    q = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = split(theta, X.shape[1], n_out)
    x = q(X)
    a1 = q(np.maximum(x @ q(W1).T + b1, 0.0))
    a2 = q(np.maximum(a1 @ q(W2).T + b2, 0.0))
    y = a2 @ q(W3).T + b3
    return y, (x, a1, a2)


def loss_and_grad(theta, X, T, rounding=True, round_deltas=True):
    """L = mean((Y - T)^2) over batch and outputs, and dL/dtheta.  With
    rounding, the forward operands are BF16 and (round_deltas) so are the
    operands of the backward products: the output gradient and the
    back-propagated deltas (BF16 mixed-precision training, see the module
    docstring); the rounding itself is differentiated as the identity."""
    n_out = T.shape[1]
    qf = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    q = qf if round_deltas else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = split(theta, X.shape[1], n_out)
    y, (x, a1, a2) = forward(theta, X, n_out, rounding)
    B = X.shape[0]
    L = np.mean((y - T) ** 2)
    dy = q(2.0 * (y - T) / (B * n_out))
    gW3 = dy.T @ a2
    gb3 = dy.sum(axis=0)
    d2 = q((dy @ qf(W3)) * (a2 > 0))
    gW2 = d2.T @ a1
    gb2 = d2.sum(axis=0)
    d1 = q((d2 @ qf(W2)) * (a1 > 0))
    gW1 = d1.T @ x
    gb1 = d1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def adam_step(theta, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new theta, m, v."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def apply(o, theta, U, R, rounding=True, D=None):
    """z = s_K * MLP(x_K) for every element, plus D_K^{-1} r_K when the blocks D
    are given (correction mode), returned as [e, c, b]."""
    X, s = features(o, U, R)
    y, _ = forward(theta, X, o.nvar * o.nb, rounding)
    z = (s[:, None] * y).reshape(o.ne, o.nvar, o.nb)
    return z if D is None else z + block_apply(D, R)
