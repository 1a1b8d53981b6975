"""TEST INFRASTRUCTURE ONLY: post-processing of top-lists (Sec. V.E), the plain CPU version.

Only the test suite may import this module.  Written from the paper's description of the three
post-processing steps:

* ``resolutions`` -- the parameter-space resolutions at a template: delta f = 1/Tc and the sky
  resolution delta Theta = c / (v Tc f P_F) of Sec. IV.C, and the binary resolutions of
  eq:binaryres (delta a_p, delta Omega, delta t_asc) with mismatch parameters m_a, m_Omega, m_t.
* ``distance2``   -- eq:postdist, the squared dimensionless distance between two templates, with
  each point-dependent resolution replaced by the mean of its values at the two templates.
* ``coincidences`` -- step 1: pairs of templates from two top-lists closer than a window, each
  replaced by its significance-weighted centroid.
* ``clusters``    -- step 2: templates closer than a window are linked and linked templates share
  a cluster; clusters that share a template are merged, i.e. the clusters are the connected
  components of the "closer than the window" graph.  Each cluster is labelled by its smallest
  member index.
* ``centroids``   -- step 2 (option B cut) and step 3: optionally drop members farther than a cut
  from the cluster's most significant member, then the significance-weighted centroid and the
  summed significance of each cluster, and the most significant cluster of the list.

Template rows are (f [Hz], x, y, a_p [lt-s], Omega [rad/s], t_asc [s]); x and y are the
projection of the sky direction on the ecliptic plane.

The window and cut decisions compare d^2 with the squared window in FP64 with this fixed
evaluation order (the GPU library takes the same decisions the same way):

    k       = (pi * Tc) * f
    dTheta  = 1 / (((v * Tc) * f) * P_F)
    da_p    = sqrt(6 m_a) / (k * Omega)
    dOmega  = sqrt(72 m_Omega) / (((k * a_p) * Omega) * T_obs)
    dt_asc  = sqrt(6 m_t) / (((k * a_p) * Omega) * Omega)
    q_f     = (f_b - f_a) * Tc,      q_z = (z_b - z_a) / ((dz_a + dz_b) * 0.5) otherwise
    d^2     = ((((q_f^2 + q_x^2) + q_y^2) + q_a^2) + q_Omega^2) + q_t^2

Readings where the paper is silent: the mean resolution is the arithmetic mean of the two
templates' resolutions; v in the sky resolution is |v|/c of the detector's orbital motion
(1e-4); t_asc differences are taken as they are (both templates sit in the orbit nearest the
mid-time); a coincident pair's significance is the sum of its two significances; the most
significant member of a cluster breaks ties by lower index, and so does the most significant
cluster of a list.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

PI = 3.141592653589793


@dataclass
class PostParams:
    t_coh: float = 900.0
    t_obs: float = 86400.0 * 120
    m_a: float = 0.4
    m_omega: float = 0.4
    m_t: float = 0.4
    pixel_factor: float = 1.0
    v_over_c: float = 1.0e-4


def resolutions(pp: PostParams, cand: np.ndarray) -> np.ndarray:
    """[n, 4]: (dTheta, da_p, dOmega, dt_asc) at each template (Sec. IV.C, eq:binaryres)."""
    c = np.asarray(cand, dtype=np.float64).reshape(-1, 6)
    f, a, W = c[:, 0], c[:, 3], c[:, 4]
    k = (PI * pp.t_coh) * f
    d_theta = 1.0 / (((pp.v_over_c * pp.t_coh) * f) * pp.pixel_factor)
    d_a = math.sqrt(6.0 * pp.m_a) / (k * W)
    d_w = math.sqrt(72.0 * pp.m_omega) / (((k * a) * W) * pp.t_obs)
    d_t = math.sqrt(6.0 * pp.m_t) / (((k * a) * W) * W)
    return np.stack([d_theta, d_a, d_w, d_t], axis=1)


def distance2(pp: PostParams, ca: np.ndarray, cb: np.ndarray, ra: Optional[np.ndarray] = None,
              rb: Optional[np.ndarray] = None) -> np.ndarray:
    """eq:postdist squared, between rows of ca and rows of cb (broadcast), mean resolutions."""
    ca = np.asarray(ca, dtype=np.float64)
    cb = np.asarray(cb, dtype=np.float64)
    ra = resolutions(pp, ca).reshape(ca.shape[:-1] + (4,)) if ra is None else ra
    rb = resolutions(pp, cb).reshape(cb.shape[:-1] + (4,)) if rb is None else rb
    qf = (cb[..., 0] - ca[..., 0]) * pp.t_coh
    qx = (cb[..., 1] - ca[..., 1]) / ((ra[..., 0] + rb[..., 0]) * 0.5)
    qy = (cb[..., 2] - ca[..., 2]) / ((ra[..., 0] + rb[..., 0]) * 0.5)
    qa = (cb[..., 3] - ca[..., 3]) / ((ra[..., 1] + rb[..., 1]) * 0.5)
    qw = (cb[..., 4] - ca[..., 4]) / ((ra[..., 2] + rb[..., 2]) * 0.5)
    qt = (cb[..., 5] - ca[..., 5]) / ((ra[..., 3] + rb[..., 3]) * 0.5)
    return ((((qf * qf + qx * qx) + qy * qy) + qa * qa) + qw * qw) + qt * qt


def distance_matrix2(pp: PostParams, ca: np.ndarray, cb: np.ndarray) -> np.ndarray:
    """[na, nb] squared distances, one row at a time."""
    ca = np.asarray(ca, dtype=np.float64).reshape(-1, 6)
    cb = np.asarray(cb, dtype=np.float64).reshape(-1, 6)
    ra, rb = resolutions(pp, ca), resolutions(pp, cb)
    out = np.empty((ca.shape[0], cb.shape[0]))
    for i in range(ca.shape[0]):
        out[i] = distance2(pp, ca[i][None, :], cb, ra[i][None, :], rb)
    return out


def coincidences(pp: PostParams, ca, sa, cb, sb, window: float):
    """Step 1: pairs (i, j), i of list a and j of list b, with d < window, in (i, j) order.

    Returns (pairs [m, 2] int64, centroid [m, 6], significance [m])."""
    ca = np.asarray(ca, dtype=np.float64).reshape(-1, 6)
    cb = np.asarray(cb, dtype=np.float64).reshape(-1, 6)
    sa = np.asarray(sa, dtype=np.float64)
    sb = np.asarray(sb, dtype=np.float64)
    d2 = distance_matrix2(pp, ca, cb)
    ii, jj = np.nonzero(d2 < window * window)          # row-major: (i, j) order
    wa, wb = sa[ii], sb[jj]
    cen = (wa[:, None] * ca[ii] + wb[:, None] * cb[jj]) / (wa + wb)[:, None]
    return np.stack([ii, jj], axis=1).astype(np.int64), cen, wa + wb


def clusters(pp: PostParams, c, window: float) -> np.ndarray:
    """Step 2: label of each template = smallest index of its connected component."""
    c = np.asarray(c, dtype=np.float64).reshape(-1, 6)
    n = c.shape[0]
    adj = distance_matrix2(pp, c, c) < window * window
    label = np.full(n, -1, dtype=np.int64)
    for s in range(n):                                 # breadth-first search from each new root
        if label[s] >= 0:
            continue
        label[s] = s
        frontier = [s]
        while frontier:
            nxt = []
            for u in frontier:
                for v in np.nonzero(adj[u] & (label < 0))[0]:
                    label[v] = s
                    nxt.append(int(v))
            frontier = nxt
    return label


def centroids(pp: PostParams, c, s, label, cut: Optional[float] = None):
    """Steps 2-3 per cluster.  Returns a dict root -> (top, members, weight, centroid) and the root
    of the most significant cluster (largest summed significance; lower root on ties)."""
    c = np.asarray(c, dtype=np.float64).reshape(-1, 6)
    s = np.asarray(s, dtype=np.float64)
    label = np.asarray(label)
    out = {}
    for r in np.unique(label):
        mem = np.nonzero(label == r)[0]
        top = int(mem[np.lexsort((mem, -s[mem]))[0]])          # largest s, then lowest index
        if cut is not None:
            d2 = distance2(pp, c[top][None, :], c[mem])
            keep = mem[(d2 < cut * cut) | (mem == top)]
        else:
            keep = mem
        wsum = 0.0
        acc = np.zeros(6)
        for m in keep:                                   # plain sums in member order
            wsum += s[m]
            acc += s[m] * c[m]
        out[int(r)] = (top, keep, wsum, acc / wsum)
    best = None
    for r in sorted(out):
        if best is None or out[r][2] > out[best][2]:
            best = r
    return out, best
