"""FP64 reference for the learned warm start: feature rows, targets, the MLP
forward / backward pass and the Adam update.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The warm start is not in the paper; it is the batched extension of the ADMM
start of Sec. IV-A (the iterate (z, y) and penalty rho that the iterations
begin from).  What is computed here:

Feature row (d_in = 160) of stage k = 0..N of a box-constrained instance
(rows [x_k; u_k] per stage, terminal rows x_N), with x_max the upper bound
of the first state row and u_max that of the first input row:
    f[0:nx]      x0 / x_max
    f[75], f[76] x_max / 5, u_max
    f[77:141]    S d_k, the 64-d linearisation sketch, with
                 d_k = [ (A_k - I) x0 (rows 0..nx-1 of a 75-slot),
                         B_k^T x0    (rows 75..75+nu-1 of a 19-slot) ] / x_max
                 and d_N = 0; S (64 x 94) is a fixed random input
    f[141:145]   k / N, N / 512, nx / 75, nu / 19
    f[145:160]   0
Target row (d_out = 192): z of the stage's state rows / x_max in [0:nx],
input rows / u_max in [75:75+nu], lambda = rho y of the state rows in
[94:94+nx], input rows in [169:169+nu], log10 of the solver's final rho in
[188]; the mask (a loss weight) is 1 on the z and lambda entries and
RHO_WEIGHT on the rho entry, 0 elsewhere.

MLP: h1 = relu(X W1 + b1), h2 = relu(h1 W2 + b2), h3 = relu(h2 W3 + b3),
Y = h3 W4 + b4, sizes 160-512-512-512-192.  Parameters are one flat vector in
the order W1 (d_in x d_out, row-major), b1, W2, b2, W3, b3, W4, b4.
Loss  L = sum(M * (Y - T)^2) / sum(M)  (M: per-entry weights).
Adam (Kingma & Ba, 2015) with bias correction:
    m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
    theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

SIZES = (160, 512, 512, 512, 192)
D_IN, D_OUT = 160, 192
XS, US = 75, 19           # state / input slots of the padded layouts
RHO_COL = 188
RHO_WEIGHT = 25.0         # loss weight of the rho entry (one entry per row vs up to 188 others)


def n_params(sizes=SIZES):
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def unflatten(theta, sizes=SIZES):
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = theta[o:o + a * b].reshape(a, b); o += a * b
        bb = theta[o:o + b]; o += b
        out.append((W, bb))
    assert o == theta.size
    return out


def forward(theta, X, sizes=SIZES):
    """Returns Y and the list of layer inputs (X, h1, h2, h3)."""
    layers = unflatten(np.asarray(theta, dtype=np.float64), sizes)
    h = np.asarray(X, dtype=np.float64)
    acts = []
    for i, (W, b) in enumerate(layers):
        acts.append(h)
        a = h @ W + b
        h = np.maximum(a, 0.0) if i + 1 < len(layers) else a
    return h, acts


def loss(theta, X, T, M, sizes=SIZES):
    Y, _ = forward(theta, X, sizes)
    return float(np.sum(M * (Y - T) ** 2) / np.sum(M))


def loss_grad(theta, X, T, M, sizes=SIZES):
    """Loss and its gradient with respect to the flat parameter vector, by
    the chain rule through the layers (reverse mode).  The back-propagated
    quantities are carried as 2 M (Y - T) and its images, and every gradient
    is divided by sum(M) at the end (the same numbers as dividing first)."""
    layers = unflatten(np.asarray(theta, dtype=np.float64), sizes)
    Y, acts = forward(theta, X, sizes)
    cnt = float(np.sum(M))
    L = float(np.sum(M * (Y - T) ** 2) / cnt)
    dA = 2.0 * M * (Y - T)                    # dL/d(pre-activation) of the last layer, times sum(M)
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        h = acts[i]
        grads.append((h.T @ dA / cnt, dA.sum(axis=0) / cnt))
        if i > 0:
            dh = dA @ W.T
            dA = dh * (h > 0.0)               # h = relu(a) of layer i-1: relu'(a) = [h > 0]
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, flat


def adam(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1).  Returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------ features

def bound_scales(p):
    """(x_max, u_max): upper bounds of the first state row and the first
    input row of stage 0."""
    return float(p.u[0]), float(p.u[p.nx])


def features(p, sketch, x0=None):
    """Feature rows [N+1, 160] of a box instance (definition in the module
    docstring)."""
    N, nx, nu = p.N, p.nx, p.nu
    x0 = p.x0 if x0 is None else np.asarray(x0, dtype=np.float64)
    xm, um = bound_scales(p)
    F = np.zeros((N + 1, D_IN))
    F[:, :nx] = x0 / xm
    F[:, 75] = xm / 5.0
    F[:, 76] = um
    for k in range(N + 1):
        d = np.zeros(XS + US)
        if k < N:
            d[:nx] = (p.A[k] @ x0 - x0) / xm
            d[XS:XS + nu] = (p.B[k].T @ x0) / xm
        F[k, 77:141] = sketch @ d
        F[k, 141] = k / N
    F[:, 142] = N / 512.0
    F[:, 143] = nx / 75.0
    F[:, 144] = nu / 19.0
    return F


def targets(p, z, lam, rho):
    """Target rows and mask [N+1, 192] from a solution (z, lambda) and the
    final rho."""
    N, nx, nu, nc = p.N, p.nx, p.nu, p.nc
    xm, um = bound_scales(p)
    T = np.zeros((N + 1, D_OUT)); M = np.zeros((N + 1, D_OUT))
    for k in range(N + 1):
        if k < N:
            zz, ll = z[k * nc:(k + 1) * nc], lam[k * nc:(k + 1) * nc]
            T[k, :nx] = zz[:nx] / xm; T[k, XS:XS + nu] = zz[nx:] / um
            T[k, 94:94 + nx] = ll[:nx]; T[k, 169:169 + nu] = ll[nx:]
            M[k, :nx] = M[k, XS:XS + nu] = M[k, 94:94 + nx] = M[k, 169:169 + nu] = 1.0
        elif p.nf:
            T[k, :nx] = z[N * nc:] / xm; T[k, 94:94 + nx] = lam[N * nc:]
            M[k, :nx] = M[k, 94:94 + nx] = 1.0
        T[k, RHO_COL] = np.log10(rho); M[k, RHO_COL] = RHO_WEIGHT
    return T, M


def warm_start(p, Y, rho_min=1e-6, rho_max=1e6):
    """The start the predicted rows give: rho0 = 10^(mean of the rho column
    over the instance's rows), clamped; z0 = the predicted z scaled back and
    projected onto [l, u]; y0 = predicted lambda / rho0."""
    N, nx, nu, nc = p.N, p.nx, p.nu, p.nc
    xm, um = bound_scales(p)
    rho = float(np.clip(10.0 ** np.mean(Y[:, RHO_COL]), rho_min, rho_max))
    z = np.zeros(p.m); lam = np.zeros(p.m)
    for k in range(N):
        z[k * nc:k * nc + nx] = Y[k, :nx] * xm
        z[k * nc + nx:(k + 1) * nc] = Y[k, XS:XS + nu] * um
        lam[k * nc:k * nc + nx] = Y[k, 94:94 + nx]
        lam[k * nc + nx:(k + 1) * nc] = Y[k, 169:169 + nu]
    if p.nf:
        z[N * nc:] = Y[N, :nx] * xm
        lam[N * nc:] = Y[N, 94:94 + nx]
    z = np.minimum(np.maximum(z, p.l), p.u)
    return z, lam / rho, rho
