"""FP64 reference of the expansion-order network and its training data.

TEST INFRASTRUCTURE ONLY: used by the tests and nothing else.  It shares no
code with the GPU path.

Network (order selection per interaction): 12 inputs -> 64 -> 64 -> 9, ReLU
after the two hidden layers, a linear output layer.  Output k predicts
log10 of the relative field error of M2L truncated at order p' = k + 2
(p' = 2..10) for one (source cell, separation) pair.  Loss: mean squared
error over all outputs of a batch.

Flat parameter vector (5577 entries, this order): W1[64][12], b1[64],
W2[64][64], b2[64], W3[9][64], b3[9] (row-major; y = W x + b per layer).

Training data for a (source multipole M, integer offset v) pair in cell
units (source cell of side 1 at the origin, target cell centred at v):
  features x[0]    = |v| / (sqrt(3)/2)   (separation / cell radius)
           x[1+n]  = log10(|M^(n)| + 1e-300) - log10(max_k |M^(k)| + 1e-300),
                     n = 0..10, |M^(n)| the 2-norm of the rank-n
                     independent components (n_z in {0,1})
  labels   y[k]    = log10(max(e(k+2), 1e-15)), where e(p') is the relative
                     2-norm difference of (phi, grad phi) at 8 points
                     (+-3/8, +-3/8, +-3/8) of the target cell between the
                     local expansions of M2L at order p' (Eq. M2L truncated
                     at |n| + |m| <= p') and at order 10, both evaluated by
                     L2P (Eq. L2P) of order 10.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 12, 64, 9
NPARAM = NH * NIN + NH + NH * NH + NH + NOUT * NH + NOUT
SAMPLE_POINTS = np.array([[sx, sy, sz] for sz in (-0.375, 0.375) for sy in (-0.375, 0.375)
                          for sx in (-0.375, 0.375)])


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == NPARAM
    o = 0
    out = []
    for shape in ((NH, NIN), (NH,), (NH, NH), (NH,), (NOUT, NH), (NOUT,)):
        k = int(np.prod(shape))
        out.append(theta[o:o + k].reshape(shape))
        o += k
    return out


def forward(theta, X):
    """Outputs Y [B, 9] and the pre-activations (Z1, Z2) for inputs X [B, 12]."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1.T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2.T + b2
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ W3.T + b3
    return Y, (X, Z1, H1, Z2, H2)


def loss(theta, X, T):
    Y, _ = forward(theta, X)
    return float(np.mean((Y - np.asarray(T, dtype=np.float64)) ** 2))


def grad(theta, X, T):
    """Gradient of loss() with respect to theta (backpropagation)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    Y, (X, Z1, H1, Z2, H2) = forward(theta, X)
    T = np.asarray(T, dtype=np.float64)
    dY = 2.0 * (Y - T) / Y.size
    gW3 = dY.T @ H2
    gb3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * (Z2 > 0.0)
    gW2 = dZ2.T @ H1
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * (Z1 > 0.0)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(axis=0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def init_params(seed):
    """He-uniform weights, zero biases (a starting point for tests)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((NIN, NH), (NH, NH), (NH, NOUT)):
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, (fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


# ------------------------------------------------------------ training data

def independent_mask(p=10):
    """Boolean mask over the oracle's full storage: components with n_z <= 1."""
    import oracle
    return np.array([m[2] <= 1 for m in oracle.multi_indices(p)])


def features(M_full, v):
    """The 12 inputs for the full-storage order-10 multipole M (cell of side
    1) and the integer offset v."""
    import oracle
    idx = oracle.multi_indices(10)
    ranks = np.array([sum(m) for m in idx])
    ind = independent_mask(10)
    norms = np.array([np.sqrt(np.sum(M_full[(ranks == n) & ind] ** 2)) for n in range(11)])
    x = np.empty(NIN)
    x[0] = np.sqrt(float(np.dot(v, v))) / (np.sqrt(3.0) / 2.0)
    x[1:] = np.log10(norms + 1e-300) - np.log10(norms.max() + 1e-300)
    return x


def truncation_labels(M_full, v):
    """The 9 labels (see the module docstring) in FP64."""
    import oracle
    v = np.asarray(v, dtype=np.float64)
    nf10 = oracle.nfull(10)
    fields = {}
    for pp in range(2, 11):
        nf = oracle.nfull(pp)
        L = np.zeros(nf10)
        L[:nf] = oracle.m2l(pp, v, M_full[:nf])
        F = []
        for u in SAMPLE_POINTS:
            phi, g = oracle.l2p(10, u, L)
            F.extend([phi, g[0], g[1], g[2]])
        fields[pp] = np.array(F)
    ref = fields[10]
    e = np.array([np.linalg.norm(fields[pp] - ref) / np.linalg.norm(ref) for pp in range(2, 11)])
    return np.log10(np.maximum(e, 1e-15))


def choose_orders(Y, target_rel_err, margin):
    """Smallest p' in 2..10 whose predicted log10 error is at most
    log10(target) - margin; 10 when none is (fixed-p fallback)."""
    thr = np.log10(target_rel_err) - margin
    Y = np.atleast_2d(Y)
    out = np.full(Y.shape[0], 10, dtype=np.int32)
    for i in range(Y.shape[0]):
        ok = np.nonzero(Y[i] <= thr)[0]
        if ok.size:
            out[i] = int(ok[0]) + 2
    return out
