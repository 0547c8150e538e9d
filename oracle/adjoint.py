"""Analytic gradients of the real-filter forms (an extension; the paper has no
backward pass). Derived directly from the definitions:

convolution   y(p) = Re sum_{k>=0} w_k sum_x M_k(p - x) F_k(x),  M_k = H e^{-i k theta}
  dL/dH(q)     = Re sum_k w_k e^{-i k theta(q)} A_k(q),  A_k(q) = sum_x gbar(q + x) F_k(x)
  dL/dtheta(q) = H(q) sum_k w_k k Im(e^{-i k theta(q)} A_k(q))
  dL/dF_k(x)   = w_k sum_p gbar(p) conj(M_k(p - x))

correlation   y(p) = Re sum_{k>=0} w_k e^{i k theta(p)} sum_x H(p + x) conj(F_k(x))
  dL/dH(q)     = Re sum_k w_k sum_p gbar(p) e^{i k theta(p)} conj(F_k(q - p))
  dL/dtheta(p) = -gbar(p) sum_k w_k k Im(e^{i k theta(p)} G_k(p))
  dL/dF_k(x)   = w_k sum_p gbar(p) e^{i k theta(p)} H(p + x)

For a complex parameter z the gradient is reported as dL/dRe z + i dL/dIm z.
Two evaluation routes: 'direct' loops over the S x S offsets (small images, and the
finite-difference checks) and 'fft' uses zero-padded transforms.
"""
from __future__ import annotations

import numpy as np

from .extended import _place, _half_weights


def _shifted(a, dy, dx):
    """b[p] = a[p + (dy, dx)] with zeros outside."""
    ny, nx = a.shape
    out = np.zeros_like(a)
    ys0, ys1 = max(0, -dy), min(ny, ny - dy)
    xs0, xs1 = max(0, -dx), min(nx, nx - dx)
    if ys0 < ys1 and xs0 < xs1:
        out[ys0:ys1, xs0:xs1] = a[ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx]
    return out


def _corr_direct(a, b, R):
    """c(x) = sum_p a(p) conj(b(p - x)) for |dx|, |dy| <= R; returns (2R+1)^2 array."""
    S = 2 * R + 1
    c = np.zeros((S, S), dtype=np.complex128)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            c[R + dy, R + dx] = np.sum(a * np.conj(_shifted(b, -dy, -dx)))
    return c


def _corr_fft(a, b, R):
    ny, nx = a.shape
    Py, Px = ny + R, nx + R
    c = np.fft.ifft2(np.fft.fft2(a, s=(Py, Px)) * np.conj(np.fft.fft2(b, s=(Py, Px))))
    idx = np.arange(-R, R + 1)
    return c[np.ix_(idx % Py, idx % Px)]


def _apply(a, Fk, conj_filter):
    """sum_x a(q + x) G(x) with G = F_k (conj_filter False) or conj(F_k) (True)."""
    S = Fk.shape[0]
    R = (S - 1) // 2
    ny, nx = a.shape
    Py, Px = ny + R, nx + R
    G = np.conj(Fk) if conj_filter else Fk
    # sum_x a(q+x) G(x) = correlation of a with conj(G)
    Gh = np.fft.fft2(_place(np.conj(G), Py, Px))
    return np.fft.ifft2(np.fft.fft2(a, s=(Py, Px)) * np.conj(Gh))[:ny, :nx]


def _scatter(a, Fk):
    """sum_q a(q) F(p - q) (plain convolution, zero boundary, same size)."""
    S = Fk.shape[0]
    R = (S - 1) // 2
    ny, nx = a.shape
    Py, Px = ny + R, nx + R
    return np.fft.ifft2(np.fft.fft2(a, s=(Py, Px)) * np.fft.fft2(_place(Fk, Py, Px)))[:ny, :nx]


def conv_backward(H, theta, comps_half, gbar, weights=None, route="fft"):
    """Gradients of the extended convolution (real-filter form) w.r.t. H, theta, F_k."""
    H = np.asarray(H, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    gbar = np.asarray(gbar, dtype=np.float64)
    comps_half = np.asarray(comps_half, dtype=np.complex128)
    U, S, _ = comps_half.shape
    R = (S - 1) // 2
    w = _half_weights(U, weights)
    gH = np.zeros_like(H)
    gT = np.zeros_like(H)
    gF = np.zeros((U, S, S), dtype=np.complex128)
    for k in range(U):
        ph = np.exp(-1j * k * theta)
        A = _apply(gbar, comps_half[k], conj_filter=False)        # A_k(q) = sum_x gbar(q+x) F_k(x)
        gH += w[k] * np.real(ph * A)
        gT += w[k] * k * np.imag(ph * A)
        Mk = H * ph
        corr = _corr_direct(gbar, Mk, R) if route == "direct" else _corr_fft(gbar, Mk, R)
        gF[k] = w[k] * corr
    return gH, H * gT, gF


def corr_backward(H, theta, comps_half, gbar, weights=None, route="fft"):
    """Gradients of the extended correlation (real-filter form) w.r.t. H, theta, F_k."""
    H = np.asarray(H, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    gbar = np.asarray(gbar, dtype=np.float64)
    comps_half = np.asarray(comps_half, dtype=np.complex128)
    U, S, _ = comps_half.shape
    R = (S - 1) // 2
    w = _half_weights(U, weights)
    gH = np.zeros_like(H)
    gT = np.zeros_like(H)
    gF = np.zeros((U, S, S), dtype=np.complex128)
    for k in range(U):
        ph = np.exp(1j * k * theta)
        gH += w[k] * np.real(_scatter(gbar * ph, np.conj(comps_half[k])))
        G = _apply(H, comps_half[k], conj_filter=True)             # G_k = H star F_k
        gT -= w[k] * k * np.imag(ph * G)
        # sum_p gbar(p) e^{ik theta(p)} H(p + x) = sum_p a(p) conj(b(p - x')) with x' = -x
        a = gbar * ph
        c = _corr_direct(a, H, R) if route == "direct" else _corr_fft(a, H, R)
        gF[k] = w[k] * c[::-1, ::-1]
    return gH, gbar * gT, gF
