"""FP64 reference of the reciprocal-space part of Ewald summation (numpy).

TEST INFRASTRUCTURE ONLY: imported by tests/; the product path never imports it, and it imports
nothing from the product.

The paper's production runs complete the short-range (real-space) Coulomb interaction with a
particle-mesh Ewald reciprocal part (section II-C, the PME kernels of Fig. 2); it prints no
formula.  Two references are here:

* ewald_recip_direct: the plain definition of the Ewald reciprocal energy of a neutral periodic
  system of point charges in a rectangular box of volume V,
      E_rec = fC / (2 pi V) sum_{m != 0} exp(-pi^2 |m|^2 / beta^2) / |m|^2 |S(m)|^2,
      S(m) = sum_j q_j exp(2 pi i m . r_j),  m = (k1 / L1, k2 / L2, k3 / L3), k integer,
  with its forces F_i = -dE_rec / dr_i, summed over every m whose Gaussian factor exceeds
  1e-16 (an O(N M) loop over wave vectors in blocks);
* pme_reference: smooth particle-mesh Ewald, the approximation the GPU path computes, in its
  own steps: charges spread onto a K1 x K2 x K3 grid with cardinal B-splines M_n of order n,
  a 3-D FFT, multiplication by the influence function
      G(m) = fC / (pi V) exp(-pi^2 |m|^2 / beta^2) / |m|^2 |b1(m1)|^2 |b2(m2)|^2 |b3(m3)|^2,
      |b(m)|^-2 = |sum_{k=0}^{n-2} M_n(k + 1) exp(2 pi i m k / K)|^2,
  (m_a taken in (-K_a/2, K_a/2]), an inverse FFT giving the grid potential phi, the energy
  1/2 sum_k Q(k) phi(k) and the forces -sum_k dQ(k)/dr_i phi(k) from the B-spline derivatives
  dM_n(x)/dx = M_{n-1}(x) - M_{n-1}(x - 1).  It converges to ewald_recip_direct as the grid is
  refined (pinned in the tests).
"""
from __future__ import annotations

import math

import numpy as np


def _box3(box):
    return np.array([box] * 3 if np.isscalar(box) else box, dtype=np.float64)


def ewald_recip_direct(x, q, box, beta, fc, tol=1e-16, block=4096):
    """Returns (E_rec, F [n][3]) by the plain sum over wave vectors."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64)
    L = _box3(box)
    V = float(np.prod(L))
    mmax = beta * math.sqrt(-math.log(tol)) / math.pi
    kmax = [int(math.ceil(mmax * L[a])) for a in range(3)]
    k1, k2, k3 = np.meshgrid(*[np.arange(-kmax[a], kmax[a] + 1) for a in range(3)], indexing="ij")
    k = np.stack([k1.ravel(), k2.ravel(), k3.ravel()], axis=1)
    m = k / L
    m2 = (m * m).sum(axis=1)
    keep = (m2 > 0.0) & (m2 <= mmax * mmax)
    m, m2 = m[keep], m2[keep]
    w = np.exp(-math.pi ** 2 * m2 / beta ** 2) / m2
    A = fc / (2.0 * math.pi * V)
    e = 0.0
    f = np.zeros_like(x)
    for s in range(0, len(m), block):
        mb, wb = m[s:s + block], w[s:s + block]
        th = 2.0 * math.pi * (x @ mb.T)            # (n, M)
        c, sn = np.cos(th), np.sin(th)
        C, S = q @ c, q @ sn                        # (M,)
        e += A * float(np.sum(wb * (C * C + S * S)))
        # F_i = 4 pi A q_i sum_m w m (C sin th_i - S cos th_i)
        g = (sn * C - c * S) * wb                   # (n, M)
        f += 4.0 * math.pi * A * q[:, None] * (g @ mb)
    return e, f


def bspline(w, n):
    """Cardinal B-spline weights M_n(w + j), j = 0 .. n-1, for fractional parts w (shape [..]),
    by the recursion M_n(x) = x/(n-1) M_{n-1}(x) + (n-x)/(n-1) M_{n-1}(x-1), M_2(x) = 1 - |x-1|;
    also the derivatives dM_n(w + j)/dx = M_{n-1}(w + j) - M_{n-1}(w + j - 1)."""
    w = np.asarray(w, dtype=np.float64)

    def M(order, xx):
        if order == 2:
            return np.where((xx >= 0.0) & (xx <= 2.0), 1.0 - np.abs(xx - 1.0), 0.0)
        return xx / (order - 1) * M(order - 1, xx) + (order - xx) / (order - 1) * M(order - 1, xx - 1.0)

    js = np.arange(n, dtype=np.float64)
    xx = w[..., None] + js
    val = M(n, xx)
    der = M(n - 1, xx) - M(n - 1, xx - 1.0)
    return val, der


def bmod2(K, n):
    """|b(m)|^2 for m = 0 .. K-1 (the B-spline Euler exponential spline moduli)."""
    Mk, _ = bspline(np.array([0.0]), n)       # M_n(0 + j), j = 0 .. n-1
    Mk = Mk[0]
    m = np.arange(K)
    den = np.zeros(K, dtype=np.complex128)
    for kk in range(n - 1):
        den += Mk[kk + 1] * np.exp(2j * math.pi * m * kk / K)
    return 1.0 / np.abs(den) ** 2


def pme_reference(x, q, box, beta, fc, grid, order):
    """Returns (E_rec, F [n][3]) of smooth PME on a grid (K1, K2, K3) with B-splines of the
    given order."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64)
    L = _box3(box)
    K = np.array(grid, dtype=np.int64)
    V = float(np.prod(L))
    n = int(order)
    u = x / L * K                                   # scaled fractional coordinates
    fl = np.floor(u)
    w = u - fl
    base = fl.astype(np.int64)
    vals, ders = [], []
    for a in range(3):
        v, d = bspline(w[:, a], n)                  # (natoms, n)
        vals.append(v)
        ders.append(d)
    # grid points of atom i along axis a: base - j (mod K)
    idx = [np.mod(base[:, a][:, None] - np.arange(n)[None, :], K[a]) for a in range(3)]
    # flat index and weight of every (atom, j1, j2, j3): arrays [natoms][n][n][n]
    flat = (idx[0][:, :, None, None] * K[1] + idx[1][:, None, :, None]) * K[2] + idx[2][:, None, None, :]
    wt = q[:, None, None, None] * vals[0][:, :, None, None] * vals[1][:, None, :, None] * vals[2][:, None, None, :]
    Q = np.zeros(int(np.prod(K)), dtype=np.float64)
    np.add.at(Q, flat.ravel(), wt.ravel())
    Q = Q.reshape(tuple(K))
    # influence function
    ms = [np.fft.fftfreq(int(K[a]), d=1.0 / K[a]) / L[a] for a in range(3)]   # m_a = k / L
    M1, M2, M3 = np.meshgrid(*ms, indexing="ij")
    msq = M1 ** 2 + M2 ** 2 + M3 ** 2
    B = bmod2(int(K[0]), n)[:, None, None] * bmod2(int(K[1]), n)[None, :, None] * bmod2(int(K[2]), n)[None, None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        G = np.where(msq > 0.0, fc / (math.pi * V) * np.exp(-math.pi ** 2 * msq / beta ** 2) / msq * B, 0.0)
    Qh = np.fft.fftn(Q)
    phi = np.real(np.fft.ifftn(G * Qh)) * float(np.prod(K))   # unnormalised inverse
    e = 0.5 * float(np.sum(Q * phi))
    p = phi.ravel()[flat]                                   # [natoms][n][n][n]
    gx = np.einsum("ia,ib,ic,iabc->i", ders[0], vals[1], vals[2], p) * K[0] / L[0]
    gy = np.einsum("ia,ib,ic,iabc->i", vals[0], ders[1], vals[2], p) * K[1] / L[1]
    gz = np.einsum("ia,ib,ic,iabc->i", vals[0], vals[1], ders[2], p) * K[2] / L[2]
    f = -q[:, None] * np.stack([gx, gy, gz], axis=1)
    return e, f
