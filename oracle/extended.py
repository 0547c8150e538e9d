"""Extended correlation and convolution: brute-force definitions and FFT route.

Brute force follows the definitions directly:
  correlation (Sec. 2.1, eq. Def-ECorr):  y(p) = sum_q H(q) conj((T(p) F)(q - p))
  convolution (Sec. 2.2, eq. Def-EConv):  y(p) = sum_q H(q) (T(q) F)(p - q)
with T(p) F = F_{theta(p)} the band-limited filter rotated by theta(p)
(decompose.rotated_filter). Boundary reading: H is zero outside the image and the
output has the image's size.

The FFT route follows Sec. 4.1: G_k = H star F_k by zero-padded FFT correlation, then
y(p) = sum_k e^{i k theta(p)} G_k(p); for convolution the signal is first multiplied
by e^{-i k theta} and the k-th product is convolved with F_k, then summed over k.
Sizes P >= N + R per axis make the circular result equal the zero-boundary one.

Components are given as the full stack k = -K..K (index k + K); nothing here assumes
the filter is real.
"""
from __future__ import annotations

import contextlib

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

from .decompose import rotated_filter

# FFT library of the FFT routes: numpy.fft (single-threaded pocketfft) by default; inside
# fft_workers(n) scipy.fft with n threads (the same algorithm, its 1D transforms spread
# over n threads). The arithmetic of the routes does not change.
_FFT_WORKERS = None


@contextlib.contextmanager
def fft_workers(n: int):
    """Runs the FFT routes on scipy.fft with `n` worker threads within the block."""
    global _FFT_WORKERS
    old = _FFT_WORKERS
    _FFT_WORKERS = int(n)
    try:
        yield
    finally:
        _FFT_WORKERS = old


def _fft2(a, s=None):
    if _FFT_WORKERS is None:
        return np.fft.fft2(a, s=s)
    import scipy.fft
    return scipy.fft.fft2(a, s=s, workers=_FFT_WORKERS)


def _ifft2(a):
    if _FFT_WORKERS is None:
        return np.fft.ifft2(a)
    import scipy.fft
    return scipy.fft.ifft2(a, workers=_FFT_WORKERS)


def min_fft_size(n: int, R: int) -> int:
    return n + R


def _phases(theta, K):
    ks = np.arange(-K, K + 1)
    return np.exp(-1j * np.multiply.outer(np.asarray(theta, dtype=np.float64), ks))


def ext_corr_brute(H, theta, comps, row_chunk=32):
    """Extended correlation by the definition (eq. Def-ECorr), pixel by pixel."""
    H = np.asarray(H, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    comps = np.asarray(comps)
    n_c, S, _ = comps.shape
    K = (n_c - 1) // 2
    R = (S - 1) // 2
    ny, nx = H.shape
    Hp = np.pad(H, R)
    win = sliding_window_view(Hp, (S, S))          # win[i, j] = H[i-R:i+R+1, j-R:j+R+1]
    flat = comps.reshape(n_c, S * S)
    y = np.zeros((ny, nx), dtype=np.complex128)
    for i0 in range(0, ny, row_chunk):
        i1 = min(ny, i0 + row_chunk)
        rot = _phases(theta[i0:i1], K) @ flat       # F_{theta(p)}(x), shape (rows, nx, S*S)
        patch = win[i0:i1].reshape(i1 - i0, nx, S * S)
        y[i0:i1] = np.sum(patch * np.conj(rot), axis=-1)
    return y


def ext_conv_brute(H, theta, comps, row_chunk=32):
    """Extended convolution by the definition (eq. Def-EConv): every source pixel q
    scatters H(q) times the filter rotated by theta(q), centred at q."""
    H = np.asarray(H, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    comps = np.asarray(comps)
    n_c, S, _ = comps.shape
    K = (n_c - 1) // 2
    R = (S - 1) // 2
    ny, nx = H.shape
    flat = comps.reshape(n_c, S * S)
    yp = np.zeros((ny + 2 * R, nx + 2 * R), dtype=np.complex128)
    for i0 in range(0, ny, row_chunk):
        i1 = min(ny, i0 + row_chunk)
        rot = (_phases(theta[i0:i1], K) @ flat).reshape(i1 - i0, nx, S, S)
        contrib = H[i0:i1, :, None, None] * rot      # H(q) F_{theta(q)}(x)
        for dy in range(S):
            for dx in range(S):
                # x = (dx - R, dy - R); lands on p = q + x, i.e. padded index q + (dy, dx)
                yp[i0 + dy:i1 + dy, dx:dx + nx] += contrib[:, :, dy, dx]
    return yp[R:R + ny, R:R + nx]


def _place(Fk, Py, Px):
    """Put an S x S component on a Py x Px torus with its centre at index (0, 0)."""
    S = Fk.shape[0]
    R = (S - 1) // 2
    out = np.zeros((Py, Px), dtype=np.complex128)
    idx = np.arange(-R, R + 1)
    out[np.ix_(idx % Py, idx % Px)] = Fk
    return out


def _sizes(shape, R, P):
    ny, nx = shape
    if P is None:
        return min_fft_size(ny, R), min_fft_size(nx, R)
    Py, Px = (P, P) if np.isscalar(P) else P
    assert Py >= ny + R and Px >= nx + R
    return Py, Px


def standard_correlations(H, comps, P=None):
    """G_k = H star F_k for every component (Sec. 4.1, "Standard Correlation")."""
    H = np.asarray(H, dtype=np.float64)
    comps = np.asarray(comps)
    S = comps.shape[1]
    R = (S - 1) // 2
    ny, nx = H.shape
    Py, Px = _sizes(H.shape, R, P)
    Hh = _fft2(H, s=(Py, Px))
    G = np.empty((comps.shape[0], ny, nx), dtype=np.complex128)
    for i, Fk in enumerate(comps):
        Fh = _fft2(_place(Fk, Py, Px))
        G[i] = _ifft2(Hh * np.conj(Fh))[:ny, :nx]
    return G


def ext_corr_fft(H, theta, comps, P=None):
    """Extended correlation by the Sec. 4.1 algorithm: y = sum_k e^{i k theta} G_k."""
    comps = np.asarray(comps)
    K = (comps.shape[0] - 1) // 2
    G = standard_correlations(H, comps, P)
    ph = np.conj(_phases(theta, K))                 # e^{+i k theta}
    return np.einsum("ijk,kij->ij", ph, G)


def ext_conv_fft(H, theta, comps, P=None):
    """Extended convolution by pre-multiplying the signal (Sec. 4.1):
    y = sum_k (H e^{-i k theta}) * F_k."""
    H = np.asarray(H, dtype=np.float64)
    comps = np.asarray(comps)
    K = (comps.shape[0] - 1) // 2
    S = comps.shape[1]
    R = (S - 1) // 2
    ny, nx = H.shape
    Py, Px = _sizes(H.shape, R, P)
    ph = _phases(theta, K)                          # e^{-i k theta}
    acc = np.zeros((Py, Px), dtype=np.complex128)
    for i, Fk in enumerate(comps):
        Mk = H * ph[..., i]
        acc += _fft2(Mk, s=(Py, Px)) * _fft2(_place(Fk, Py, Px))
    return _ifft2(acc)[:ny, :nx]


def _half_weights(n_half, weights):
    if weights is None:
        w = np.full(n_half, 2.0)
        w[0] = 1.0
        return w
    return np.asarray(weights, dtype=np.float64)


def ext_corr_half(H, alpha, comps_half, weights=None, P=None):
    """Real-filter form of the correlation: y = Re sum_{k>=0} w_k e^{i k alpha} G_k,
    w_0 = 1, w_k = 2 (the k and -k terms are complex conjugates when F is real)."""
    comps_half = np.asarray(comps_half)
    w = _half_weights(comps_half.shape[0], weights)
    G = standard_correlations(H, comps_half, P)
    alpha = np.asarray(alpha, dtype=np.float64)
    y = np.zeros(G.shape[1:])
    for k in range(G.shape[0]):
        y += w[k] * np.real(np.exp(1j * k * alpha) * G[k])
    return y


def ext_conv_half(H, alpha, comps_half, weights=None, P=None):
    """Real-filter form of the convolution: y = Re sum_{k>=0} w_k (H e^{-i k alpha}) * F_k."""
    H = np.asarray(H, dtype=np.float64)
    comps_half = np.asarray(comps_half)
    w = _half_weights(comps_half.shape[0], weights)
    S = comps_half.shape[1]
    R = (S - 1) // 2
    ny, nx = H.shape
    Py, Px = _sizes(H.shape, R, P)
    alpha = np.asarray(alpha, dtype=np.float64)
    acc = np.zeros((Py, Px), dtype=np.complex128)
    for k, Fk in enumerate(comps_half):
        Mk = H * np.exp(-1j * k * alpha)
        acc += w[k] * _fft2(Mk, s=(Py, Px)) * _fft2(_place(Fk, Py, Px))
    return np.real(_ifft2(acc)[:ny, :nx])


def match_rotations(H, comps, n_angles=64, P=None):
    """Rotation-independent matching: response at every angle 2 pi m / A,
    C(p, m) = Re sum_k e^{i k 2 pi m / A} G_k(p) (the extended correlation with a
    constant field theta = 2 pi m / A), best score = max over m, index = the
    smallest maximising m. This is the band-limited form of taking the maximum
    over rotated-filter responses (Sec. 5.2)."""
    comps = np.asarray(comps)
    K = (comps.shape[0] - 1) // 2
    G = standard_correlations(H, comps, P)
    ks = np.arange(-K, K + 1)
    ang = 2.0 * np.pi * np.arange(n_angles) / n_angles
    E = np.exp(1j * np.outer(ang, ks))               # (A, 2K+1)
    C = np.real(np.tensordot(E, G, axes=1))          # (A, ny, nx)
    idx = np.argmax(C, axis=0)
    return C.max(axis=0), idx.astype(np.int32), C
