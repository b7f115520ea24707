"""Small crafted inputs shared by the oracle pins and the GPU parity tests."""
import dataclasses

import numpy as np

import cases


def block_case(dim=2, n_side=12, dp=0.1, jitter=0.0, seed=0, walls=False,
               turbulence=0, obc_mode=4, buffers=(), nu_l=1e-2, name="block"):
    """Lattice block [0, n_side dp]^dim of fluid particles (optionally
    jittered), optionally with 3 wall layers below y = 0."""
    P = cases.base_params(dim, dp, nu_l=nu_l, turbulence=turbulence,
                          obc_mode=obc_mode, seed=seed)
    ax = (np.arange(n_side) + 0.5) * dp
    grids = np.meshgrid(*([ax] * dim), indexing="ij")
    pts = np.zeros((grids[0].size, 3))
    for k in range(dim):
        pts[:, k] = grids[k].ravel()
    rng = np.random.default_rng(seed)
    if jitter:
        pts[:, :dim] += jitter * dp * rng.uniform(-1, 1, (pts.shape[0], dim))
    wall = np.zeros((0, 3))
    if walls:
        wx = (np.arange(-4, n_side + 4) + 0.5) * dp
        wy = -(np.arange(3) + 0.5) * dp
        if dim == 2:
            W = np.meshgrid(wx, wy, indexing="ij")
            wall = np.zeros((W[0].size, 3))
            wall[:, 0], wall[:, 1] = W[0].ravel(), W[1].ravel()
        else:
            W = np.meshgrid(wx, wy, wx, indexing="ij")
            wall = np.zeros((W[0].size, 3))
            wall[:, 0], wall[:, 1], wall[:, 2] = (W[0].ravel(), W[1].ravel(),
                                                  W[2].ravel())
    c = cases._assemble(name, P, list(buffers), pts, wall, 1,
                        k0=1e-3 if turbulence else 0.0,
                        eps0=1e-3 if turbulence else 0.0)
    return c


def with_state(case, x=None, v=None, rho=None, k=None, eps=None, tag=None):
    c = dataclasses.replace(case)
    for name, val in (("x", x), ("v", v), ("rho", rho), ("k", k),
                      ("eps", eps), ("tag", tag)):
        if val is not None:
            setattr(c, name, np.array(val, dtype=getattr(case, name).dtype))
    return c


def interior_mask(x, lo, hi, margin):
    m = np.ones(x.shape[0], dtype=bool)
    for k in range(len(lo)):
        m &= (x[:, k] > lo[k] + margin) & (x[:, k] < hi[k] - margin)
    return m


def rel_err(a, b, scale):
    """max_i |a_i - b_i| / scale_i (componentwise norms per particle)."""
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    d = np.linalg.norm(a - b, axis=1)
    return float(np.max(d / scale)) if d.size else 0.0
