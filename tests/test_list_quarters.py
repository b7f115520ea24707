"""The row trim of the list scan (host arithmetic, no GPU).

The cell build orders each cell by quarter along x; the scan of a stencil
row leaves out the quarters of the row's outer cells whose members lie
farther than the list's cap along x.  From particle i's cell-relative x
(FP32, as the scan computes it) it keeps quarters below
k_hi = ceil((r_q + x_i - cs/2) / (cs/4)) of the cell at +1 and from
k_lo = floor((x_i + 3 cs/2 - r_q) / (cs/4)) on of the cell at -1, with r_q
the cap widened by 1e-5.  A member of a left-out quarter (its quarter
found in FP64, as the cell build finds it) must lie at least the cap away
along x; on average 2.25 of the row's 3 cells remain.
"""
import numpy as np


def _quarter(rel, cs):
    return np.clip(np.floor((rel + 0.5 * cs) * (4.0 / cs)).astype(np.int64), 0, 3)


def _trim(xi, cs, rl):
    f = np.float32
    q_rl, q_w, csz = f(rl * (1 + 1e-5)), f(4.0 / cs), f(cs)
    xf = xi.astype(np.float32)
    k_hi = np.clip(np.ceil((q_rl + xf - f(0.5) * csz) * q_w).astype(np.int64), 0, 4)
    k_lo = np.clip(np.floor((xf + f(1.5) * csz - q_rl) * q_w).astype(np.int64), 0, 4)
    return k_lo, k_hi


def test_left_out_quarters_lie_beyond_the_cap():
    rng = np.random.default_rng(7)
    for h in (0.0065, 0.0125, 0.1, 1.0):
        cs = 2.6 * h
        rl = cs * (1 + 2e-6)
        xi = rng.uniform(-0.5 * cs, 0.5 * cs, 4000)
        xi[:4] = [-0.5 * cs, np.nextafter(0.5 * cs, 0.0), 0.0, -0.25 * cs]
        xj = rng.uniform(-0.5 * cs, 0.5 * cs, 3000)
        xj[:3] = [-0.5 * cs, 0.0, np.nextafter(0.5 * cs, 0.0)]
        k_lo, k_hi = _trim(xi, cs, rl)
        qj = _quarter(xj, cs)
        # the cell at +1: members in quarters >= k_hi; at -1: below k_lo
        gone_hi = qj[None, :] >= k_hi[:, None]
        d_hi = cs + xj[None, :] - xi[:, None]
        assert not np.any(gone_hi & (d_hi < rl))
        gone_lo = qj[None, :] < k_lo[:, None]
        d_lo = cs + xi[:, None] - xj[None, :]
        assert not np.any(gone_lo & (d_lo < rl))
        kept = k_hi / 4.0 + 1.0 + (4 - k_lo) / 4.0
        assert abs(kept.mean() - 2.25) < 0.02
