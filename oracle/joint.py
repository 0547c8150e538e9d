"""Joint rotation and scale fields (future work in the Conclusion: components indexed by an
angular frequency k and a log-radial frequency omega_l, phase e^{ik theta} e^{i omega_l ln s}).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The transformation at a pixel rotates the filter by theta and scales it by s:
(T F)(x) = F(R_{-theta} x / s). In log-polar coordinates (u = ln r, phi) that is a shift
by (ln s, theta), so a filter written as a sum of modes e^{i k phi} e^{i omega_l (u - u_lo)}
is transformed by multiplying mode (k, l) by e^{-i k theta} e^{-i omega_l ln s}: the
representation-theoretic construction of Sec. 4 with the product group. Readings (the
paper gives only the idea):

  J1  transformation: (T_{theta,s} F)(x) = F(R_{-theta} x / s), natural log;
  J2  modes: F_{k,l}(x) = c_{k,l} e^{i k phi(x)} e^{i omega_l (ln|x| - u_lo)} on the disk
      0 < |x| <= R (R = (S-1)/2), k = -K..K, l = -(n-1)/2..(n-1)/2 (n odd, so no Nyquist
      term), omega_l = 2 pi l / L; the centre is fixed by every transformation:
      F_{k,l}(0) = delta_k0 delta_l0 F(0);
  J3  c_{k,l}: F sampled bilinearly (zero outside the array and outside the disk) on the
      log-polar grid r_j = e^{u_lo + j L / n}, phi_m = 2 pi m / M; the angular DFT over m
      gives f_k(r_j); the n-point DFT over j of h_k(u_j) gives c_{k,l};
  J4  period: the range of ln|x| - ln s met on the grid, [u_lo, u_hi] =
      [-ln s_max, ln R - ln s_min], times period_factor; on (u_hi, u_lo + L) h_k blends
      from h_k(u_hi) back to h_k(u_lo) with a raised cosine (the scale group's S4 for
      every angular frequency); radii up to R + 1e-9 count as inside the disk and samples
      up to u_hi + 1e-12 as inside the range (so that e^{ln R} rounding above R changes
      nothing);
  J5  real filters: F_{-k,-l} = conj F_{k,l}; the half set {(0, l >= 0)} and {(k >= 1, all l)}
      with weights 1 for (0, 0) and 2 otherwise;
  J6  normalised smoothing: as the scale group, {H / s^2} over {1 / s^2}.

parity unpinned: the c_{k,l} values are defined only by J1-J6 (no closed form to compare
with); the tests pin what is exact (constant fields reduce to a textbook convolution with
the transformed filter, brute force = the FFT route, quarter-turn equivariance, constant
signals preserved by the ratio).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .decompose import bilinear


@dataclass(frozen=True)
class JointParams:
    K: int = 4                 # angular band limit: k = -K..K
    n_log: int = 9             # log-radial modes (odd)
    s_min: float = 1.0
    s_max: float = 2.0
    period_factor: float = 1.5
    M: int = 0                 # angular samples; 0 = smallest power of two >= max(8 (2K+1), 4 ceil(2 pi R))


def _M(p: JointParams, R: int) -> int:
    if p.M:
        return p.M
    need = max(8 * (2 * p.K + 1), 4 * int(np.ceil(2 * np.pi * R)))
    M = 1
    while M < need:
        M *= 2
    return M


def joint_geometry(p: JointParams, S: int):
    """(R, u_lo, u_hi, L, omega_1)."""
    R = (S - 1) // 2
    u_lo = -np.log(p.s_max)
    u_hi = np.log(R) - np.log(p.s_min)
    L = p.period_factor * (u_hi - u_lo)
    return R, u_lo, u_hi, L, 2.0 * np.pi / L


def joint_coefficients(F, p: JointParams):
    """c[k + K, l + (n-1)/2] for k = -K..K, l = -(n-1)/2..(n-1)/2 (J3, J4)."""
    F = np.asarray(F, dtype=np.float64)
    S = F.shape[0]
    assert F.shape == (S, S) and S % 2 == 1 and p.n_log % 2 == 1
    R, u_lo, u_hi, L, _ = joint_geometry(p, S)
    M, n, K = _M(p, R), p.n_log, p.K
    phi = 2.0 * np.pi * np.arange(M) / M
    uj = u_lo + np.arange(n) * L / n
    ks = np.arange(-K, K + 1)

    def f_k(u):
        """angular Fourier coefficients of F on the circle of radius e^u (zero beyond R)."""
        r = np.exp(u)
        if r > R + 1e-9:          # outside the disk (the tolerance absorbs e^{ln R} != R)
            return np.zeros(2 * K + 1, dtype=np.complex128)
        v = bilinear(F, r * np.cos(phi), r * np.sin(phi))
        return np.array([np.sum(v * np.exp(-1j * k * phi)) / M for k in ks])

    f_hi, f_lo = f_k(u_hi), f_k(u_lo)
    H = np.zeros((n, 2 * K + 1), dtype=np.complex128)
    for j, u in enumerate(uj):
        if u <= u_hi + 1e-12:     # (at u_hi both branches give f_k(e^{u_hi}))
            H[j] = f_k(u)
        else:
            t = (u - u_hi) / (u_lo + L - u_hi)
            H[j] = f_hi + (f_lo - f_hi) * 0.5 * (1.0 - np.cos(np.pi * t))
    ls = np.arange(-(n - 1) // 2, (n - 1) // 2 + 1)
    c = np.zeros((2 * K + 1, n), dtype=np.complex128)
    for a, l in enumerate(ls):
        e = np.exp(-2j * np.pi * np.arange(n) * l / n)
        c[:, a] = (e[:, None] * H).sum(axis=0) / n
    return c


def joint_components(F, p: JointParams):
    """Half set (J5): (ks, ls, weights, comps[U, S, S]) in the order k = 0 with l = 0..(n-1)/2,
    then k = 1..K with l = -(n-1)/2..(n-1)/2."""
    F = np.asarray(F, dtype=np.float64)
    S = F.shape[0]
    R, u_lo, _, _, om1 = joint_geometry(p, S)
    c = joint_coefficients(F, p)
    K, h = p.K, (p.n_log - 1) // 2
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1]
    r2 = xx * xx + yy * yy
    inside = (r2 > 0) & (r2 <= R * R)
    u = 0.5 * np.log(np.maximum(r2, 1)) - u_lo
    ph = np.arctan2(yy, xx)
    ks, ls, ws, comps = [], [], [], []
    for k in range(K + 1):
        for l in (range(0, h + 1) if k == 0 else range(-h, h + 1)):
            comp = np.where(inside, c[k + K, l + h] * np.exp(1j * k * ph) * np.exp(1j * om1 * l * u), 0.0)
            if k == 0 and l == 0:
                comp[R, R] = F[R, R]
            ks.append(k)
            ls.append(l)
            ws.append(1.0 if (k == 0 and l == 0) else 2.0)
            comps.append(comp)
    return np.array(ks), np.array(ls), np.array(ws), np.array(comps)


def joint_filter_at(F, p: JointParams, theta: float, s: float):
    """The band-limited filter rotated by theta and scaled by s (real S x S)."""
    ks, ls, ws, comps = joint_components(F, p)
    _, _, _, _, om1 = joint_geometry(p, F.shape[0])
    ph = np.exp(-1j * (ks * theta + om1 * ls * np.log(s)))
    return np.real(np.tensordot(ws * ph, comps, axes=1))


def joint_conv_brute(H, theta, s, F, p: JointParams, normalize_signal=False):
    """Extended convolution by the definition (eq. Def-EConv): every pixel q scatters
    H(q) (divided by s(q)^2 if normalize_signal) times the filter transformed by
    (theta(q), s(q)), the real part of the half-set sum (J5)."""
    H = np.asarray(H, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    ks, ls, ws, comps = joint_components(F, p)
    S = comps.shape[1]
    R = (S - 1) // 2
    _, _, _, _, om1 = joint_geometry(p, S)
    ny, nx = H.shape
    Hn = H / s ** 2 if normalize_signal else H
    yp = np.zeros((ny + 2 * R, nx + 2 * R))
    flat = comps.reshape(len(ks), S * S)
    for i in range(ny):
        ph = np.exp(-1j * (np.multiply.outer(theta[i], ks) + om1 * np.multiply.outer(np.log(s[i]), ls)))
        rot = np.real((ph * ws) @ flat).reshape(nx, S, S)      # filter at every pixel of the row
        contrib = Hn[i][:, None, None] * rot
        for j in range(nx):
            yp[i:i + S, j:j + S] += contrib[j]
    return yp[R:R + ny, R:R + nx]


def joint_conv_fft(H, theta, s, F, p: JointParams, normalize_signal=False):
    """Sec. 4.1 route with the joint phase: y = Re sum_c w_c (Hn e^{-i(k_c theta +
    omega_{l_c} ln s)}) * F_c, zero-padded FFTs at P = n + R per axis."""
    H = np.asarray(H, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    ks, ls, ws, comps = joint_components(F, p)
    S = comps.shape[1]
    R = (S - 1) // 2
    _, _, _, _, om1 = joint_geometry(p, S)
    ny, nx = H.shape
    Py, Px = ny + R, nx + R
    Hn = H / s ** 2 if normalize_signal else H
    acc = np.zeros((Py, Px), dtype=np.complex128)
    idx = np.arange(-R, R + 1)
    for k, l, w, comp in zip(ks, ls, ws, comps):
        m = Hn * np.exp(-1j * (k * theta + om1 * l * np.log(s)))
        placed = np.zeros((Py, Px), dtype=np.complex128)
        placed[np.ix_(idx % Py, idx % Px)] = comp
        acc += w * np.fft.fft2(m, s=(Py, Px)) * np.fft.fft2(placed)
    return np.real(np.fft.ifft2(acc)[:ny, :nx])


def joint_smooth(H, theta, s, F, p: JointParams, route="fft"):
    """Normalised smoothing (J6): {H / s^2} * F over {1 / s^2} * F."""
    f = joint_conv_fft if route == "fft" else joint_conv_brute
    num = f(H, theta, s, F, p, normalize_signal=True)
    den = f(np.ones_like(np.asarray(H, dtype=np.float64)), theta, s, F, p, normalize_signal=True)
    return num / den, num, den
