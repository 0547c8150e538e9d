// Generic complex transforms (float32 / float64) and the float64 filter-plan kernels:
// polar resampling + angular DFT of a filter (Sec. 4.1, "Filter Decomposition"),
// log-radial components of the scale group (Sec. 8), precision conversions.
#include "kcommon.hpp"

namespace ecc {

// ---------------------------------------------------------------------------------
// generic complex transforms with circular placement:
//   rows: buf[(j + shift_in) mod P] = in[r][j] for j < nvalid; out[r][i] = buf[(i + shift_out) mod P]
//   cols: the same along columns of B adjacent columns.
// The kernels take both shifts reduced to [0, P) by their launchers, so that the index of
// every element is one conditional add or subtract (an integer modulo by the runtime
// length would dominate the instruction count of these memory-bound passes).
constexpr int kLoadGroup = 8;

template <typename T, int NB, int DIR>
__global__ void __launch_bounds__(512) k_fft_rows(const cx<T>* __restrict__ in, long long planeIn,
                                                 int ldIn, int nrows, int nvalid, int shift_in,
                                                 cx<T>* __restrict__ out, long long planeOut,
                                                 int ldOut, int nstore, int shift_out, FftDesc d,
                                                 const cx<T>* __restrict__ tw, int B, int TF) {
  extern __shared__ char smem_raw[];
  cx<T>* twl = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = twl + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int P = d.P;
  const int c = threadIdx.x / TF, f = threadIdx.x - c * TF;
  const int row = blockIdx.x * B + c;
  const bool active = (c < B) && (row < nrows);
  Layout L{B, 0, P};
  if (active) {
    const cx<T>* src = in + (long long)blockIdx.y * planeIn + (long long)row * ldIn;
    // loads in groups of kLoadGroup per thread, all issued before their LDS stores, so that
    // several loads per thread are in flight at once
    for (int pos0 = f; pos0 < P; pos0 += kLoadGroup * TF) {
      cx<T> v[kLoadGroup];
#pragma unroll
      for (int u = 0; u < kLoadGroup; ++u) {
        const int pos = pos0 + u * TF;
        int j = pos - shift_in;
        if (j < 0) j += P;
        v[u].re = T(0);
        v[u].im = T(0);
        if (pos < P && j < nvalid) v[u] = src[j];
      }
#pragma unroll
      for (int u = 0; u < kLoadGroup; ++u)
        if (pos0 + u * TF < P) buf[c * P + pos0 + u * TF] = v[u];
    }
  }
  __syncthreads();
  run_fft<NB, DIR, false, T>(buf, L, d, twl, c, f, TF, active);
  if (active) {
    cx<T>* dst = out + (long long)blockIdx.y * planeOut + (long long)row * ldOut;
    for (int i = f; i < nstore; i += TF) {
      int pos = i + shift_out;
      if (pos >= P) pos -= P;
      dst[i] = buf[c * P + pos];
    }
  }
}

template <typename T, int NB, int DIR>
__global__ void __launch_bounds__(512) k_fft_cols(const cx<T>* __restrict__ in, long long planeIn,
                                                 int ldIn, int ncols, int nvalid, int shift_in,
                                                 cx<T>* __restrict__ out, long long planeOut,
                                                 int ldOut, int nstore, int shift_out, FftDesc d,
                                                 const cx<T>* __restrict__ tw, int lgB,
                                                 const cx<T>* __restrict__ mul) {
  extern __shared__ char smem_raw[];
  cx<T>* twl = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = twl + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int B = 1 << lgB, P = d.P, nthr = blockDim.x, TF = nthr >> lgB;
  const int c = threadIdx.x & (B - 1), f = threadIdx.x >> lgB;
  const int v0 = blockIdx.x * B;
  const cx<T>* src = in + (long long)blockIdx.y * planeIn;
  // loads in groups of kLoadGroup per thread (see k_fft_rows)
  for (int e0 = threadIdx.x; e0 < P * B; e0 += kLoadGroup * nthr) {
    cx<T> val[kLoadGroup];
#pragma unroll
    for (int u = 0; u < kLoadGroup; ++u) {
      const int e = e0 + u * nthr;
      const int pos = e >> lgB, v = v0 + (e & (B - 1));
      int j = pos - shift_in;
      if (j < 0) j += P;
      val[u].re = T(0);
      val[u].im = T(0);
      if (e < P * B && j < nvalid && v < ncols) {
        val[u] = src[(long long)j * ldIn + v];
        if (mul) val[u] = cmul(val[u], mul[(long long)j * ldIn + v]);
      }
    }
#pragma unroll
    for (int u = 0; u < kLoadGroup; ++u)
      if (e0 + u * nthr < P * B) buf[e0 + u * nthr] = val[u];
  }
  __syncthreads();
  Layout L{B, lgB, 0};
  run_fft<NB, DIR, true, T>(buf, L, d, twl, c, f, TF, true);
  cx<T>* dst = out + (long long)blockIdx.y * planeOut;
  for (int e = threadIdx.x; e < nstore * B; e += nthr) {
    const int i = e >> lgB, v = v0 + (e & (B - 1));
    if (v >= ncols) continue;
    int pos = i + shift_out;
    if (pos >= P) pos -= P;
    dst[(long long)i * ldOut + v] = buf[(pos << lgB) + (e & (B - 1))];
  }
}

// ---------------------------------------------------------------------------------
// filter decomposition (float64): bilinear polar samples on each distinct grid radius,
// angular DFT f_k(rho) = (1/M) sum_m F(rho cos phi_m, rho sin phi_m) e^{-i k phi_m}.
__device__ double bilinear64(const float* F, int S, double dx, double dy) {
  const int R = (S - 1) / 2;
  const double col = dx + R, row = dy + R;
  const double c0f = floor(col), r0f = floor(row);
  const int c0 = (int)c0f, r0 = (int)r0f;
  const double fc = col - c0f, fr = row - r0f;
  double acc = 0.0;
  for (int a = 0; a < 2; ++a) {
    const int rr = r0 + a;
    const double wr = a ? fr : 1.0 - fr;
    if (rr < 0 || rr >= S) continue;
    for (int b = 0; b < 2; ++b) {
      const int cc = c0 + b;
      const double wc = b ? fc : 1.0 - fc;
      if (cc < 0 || cc >= S) continue;
      acc += wr * wc * (double)F[rr * S + cc];
    }
  }
  return acc;
}

__global__ void __launch_bounds__(256) k_polar_dft(const float* __restrict__ F, int S, int K, int M,
                                                  const int* __restrict__ d2list,
                                                  cx<double>* __restrict__ fk) {
  extern __shared__ double smem_d[];
  double* v = smem_d;           // M samples
  double* ct = v + M;           // cos(2 pi t / M)
  double* st = ct + M;          // sin(2 pi t / M)
  const int ri = blockIdx.x;
  const double rho = sqrt((double)d2list[ri]);
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)M, &sn, &cs);
    ct[m] = cs;
    st[m] = sn;
    v[m] = bilinear64(F, S, rho * cs, rho * sn);
  }
  __syncthreads();
  for (int k = threadIdx.x; k <= K; k += blockDim.x) {
    double re = 0.0, im = 0.0;
    int t = 0;
    for (int m = 0; m < M; ++m) {
      re += v[m] * ct[t];
      im -= v[m] * st[t];
      t += k;
      if (t >= M) t -= M;
    }
    cx<double> r;
    r.re = re / (double)M;
    r.im = im / (double)M;
    fk[(long long)ri * (K + 1) + k] = r;
  }
}

// F_k(x) = f_k(|x|) e^{i k phi(x)} on the disk, F_0(0) = F(0), zero elsewhere.
__global__ void k_synth_rotation(const float* __restrict__ F, int S, int K,
                                 const int* __restrict__ rmap, const cx<double>* __restrict__ fk,
                                 cx<double>* __restrict__ comps) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = S * S;
  if (idx >= (K + 1) * n) return;
  const int k = idx / n, p = idx - k * n;
  const int R = (S - 1) / 2;
  const int dy = p / S - R, dx = p % S - R;
  cx<double> out;
  out.re = 0.0;
  out.im = 0.0;
  const int ri = rmap[p];
  if (dx == 0 && dy == 0) {
    if (k == 0) out.re = (double)F[p];
  } else if (ri >= 0) {
    const cx<double> f = fk[(long long)ri * (K + 1) + k];
    double sn, cs;
    sincos((double)k * atan2((double)dy, (double)dx), &sn, &cs);
    out.re = f.re * cs - f.im * sn;
    out.im = f.re * sn + f.im * cs;
  }
  comps[idx] = out;
}

// Scale group: h(u) = g(e^u) on [u_lo, u_hi], raised-cosine return to g(e^{u_lo}) on the
// rest of the period L; n-point DFT c_k; F_k(x) = c_k e^{i omega_k (ln|x| - u_lo)},
// k = 0..n/2 (Nyquist as a real coefficient), F_0(0) = g(0).
__global__ void __launch_bounds__(256) k_scale_components(double sigma0, double u_lo, double u_hi,
                                                         double L, int n, int R,
                                                         cx<double>* __restrict__ comps) {
  __shared__ double h[512];
  __shared__ double cre[257], cim[257];
  const int U = n / 2 + 1;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double u = u_lo + (double)j * L / (double)n;
    double val;
    if (u <= u_hi) {
      const double r = exp(u);
      val = exp(-r * r / (2.0 * sigma0 * sigma0));
    } else {
      const double rh = exp(u_hi), rl = exp(u_lo);
      const double ghi = exp(-rh * rh / (2.0 * sigma0 * sigma0));
      const double glo = exp(-rl * rl / (2.0 * sigma0 * sigma0));
      const double t = (u - u_hi) / (L - (u_hi - u_lo));
      val = ghi + (glo - ghi) * 0.5 * (1.0 - cospi(t));
    }
    h[j] = val;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < U; k += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int j = 0; j < n; ++j) {
      double sn, cs;
      sincospi(2.0 * (double)((long long)j * k % n) / (double)n, &sn, &cs);
      re += h[j] * cs;
      im -= h[j] * sn;
    }
    re /= (double)n;
    im /= (double)n;
    if (2 * k == n) im = 0.0;   // Nyquist coefficient is real for real h
    cre[k] = re;
    cim[k] = im;
  }
  __syncthreads();
  const int S = 2 * R + 1;
  for (int idx = threadIdx.x; idx < U * S * S; idx += blockDim.x) {
    const int k = idx / (S * S), p = idx - k * S * S;
    const int dy = p / S - R, dx = p % S - R;
    const int r2 = dx * dx + dy * dy;
    cx<double> out;
    out.re = 0.0;
    out.im = 0.0;
    if (r2 == 0) {
      if (k == 0) out.re = 1.0;   // g(0)
    } else if (r2 <= R * R) {
      const double ph = 2.0 * kPi * (double)k / L * (0.5 * log((double)r2) - u_lo);
      double sn, cs;
      sincos(ph, &sn, &cs);
      out.re = cre[k] * cs - cim[k] * sn;
      out.im = cre[k] * sn + cim[k] * cs;
    }
    comps[idx] = out;
  }
}

__global__ void k_d2f(const cx<double>* __restrict__ in, cx<float>* __restrict__ out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = mk((float)in[i].re, (float)in[i].im);
}
__global__ void k_conj_d(const cx<double>* __restrict__ in, cx<double>* __restrict__ out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = conj(in[i]);
}
__global__ void k_scale_f(float* __restrict__ y, long long n, float a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] *= a;
}
__global__ void k_f2d(const cx<float>* __restrict__ in, cx<double>* __restrict__ out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    cx<double> r;
    r.re = in[i].re;
    r.im = in[i].im;
    out[i] = r;
  }
}


// ---------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------
// host launchers
size_t lds_rows(const RowCfg& c, const FftDesc& d, size_t elem) {
  return elem * ((size_t)((d.twsize + 1) & ~1) + (size_t)c.B * d.P);
}
size_t lds_cols(const ColCfg& c, const FftDesc& d, size_t elem) {
  return elem * ((size_t)((d.twsize + 1) & ~1) + ((size_t)d.P << c.lgB));
}


template <typename T>
hipError_t launch_fft_rows(hipStream_t s, const RowCfg& c, int nplanes, int dir, const cx<T>* in,
                           long long planeIn, int ldIn, int nrows, int nvalid, int shift_in,
                           cx<T>* out, long long planeOut, int ldOut, int nstore, int shift_out,
                           const FftDesc& d, const cx<T>* tw) {
  if (nstore > d.P || nvalid > d.P) return hipErrorInvalidValue;
  shift_in = ((shift_in % d.P) + d.P) % d.P;
  shift_out = ((shift_out % d.P) + d.P) % d.P;
  if (c.B * c.TF > 512) return hipErrorInvalidValue;   // the kernel's launch bound
  dim3 grid((nrows + c.B - 1) / c.B, nplanes), block(c.B * c.TF);
  const size_t lds = lds_rows(c, d, sizeof(cx<T>));
  if (dir < 0) {
    ECC_NB_SWITCH(c.NB, hipLaunchKernelGGL((k_fft_rows<T, NB, -1>), grid, block, lds, s, in, planeIn,
                                           ldIn, nrows, nvalid, shift_in, out, planeOut, ldOut,
                                           nstore, shift_out, d, tw, c.B, c.TF));
  } else {
    ECC_NB_SWITCH(c.NB, hipLaunchKernelGGL((k_fft_rows<T, NB, +1>), grid, block, lds, s, in, planeIn,
                                           ldIn, nrows, nvalid, shift_in, out, planeOut, ldOut,
                                           nstore, shift_out, d, tw, c.B, c.TF));
  }
  return last();
}

template <typename T>
hipError_t launch_fft_cols(hipStream_t s, const ColCfg& c, int nplanes, int dir, const cx<T>* in,
                           long long planeIn, int ldIn, int ncols, int nvalid, int shift_in,
                           cx<T>* out, long long planeOut, int ldOut, int nstore, int shift_out,
                           const FftDesc& d, const cx<T>* tw, const cx<T>* mul) {
  if (nstore > d.P || nvalid > d.P) return hipErrorInvalidValue;
  shift_in = ((shift_in % d.P) + d.P) % d.P;
  shift_out = ((shift_out % d.P) + d.P) % d.P;
  const int B = 1 << c.lgB;
  dim3 grid((ncols + B - 1) / B, nplanes), block(c.nthr);
  const size_t lds = lds_cols(c, d, sizeof(cx<T>));
  if (dir < 0) {
    ECC_NB_SWITCH(c.NB, hipLaunchKernelGGL((k_fft_cols<T, NB, -1>), grid, block, lds, s, in, planeIn,
                                           ldIn, ncols, nvalid, shift_in, out, planeOut, ldOut,
                                           nstore, shift_out, d, tw, c.lgB, mul));
  } else {
    ECC_NB_SWITCH(c.NB, hipLaunchKernelGGL((k_fft_cols<T, NB, +1>), grid, block, lds, s, in, planeIn,
                                           ldIn, ncols, nvalid, shift_in, out, planeOut, ldOut,
                                           nstore, shift_out, d, tw, c.lgB, mul));
  }
  return last();
}

template hipError_t launch_fft_rows<float>(hipStream_t, const RowCfg&, int, int, const cx<float>*,
                                           long long, int, int, int, int, cx<float>*, long long, int,
                                           int, int, const FftDesc&, const cx<float>*);
template hipError_t launch_fft_rows<double>(hipStream_t, const RowCfg&, int, int, const cx<double>*,
                                            long long, int, int, int, int, cx<double>*, long long,
                                            int, int, int, const FftDesc&, const cx<double>*);
template hipError_t launch_fft_cols<float>(hipStream_t, const ColCfg&, int, int, const cx<float>*,
                                           long long, int, int, int, int, cx<float>*, long long, int,
                                           int, int, const FftDesc&, const cx<float>*, const cx<float>*);
template hipError_t launch_fft_cols<double>(hipStream_t, const ColCfg&, int, int, const cx<double>*,
                                            long long, int, int, int, int, cx<double>*, long long,
                                            int, int, int, const FftDesc&, const cx<double>*, const cx<double>*);

hipError_t launch_polar_dft(hipStream_t s, const float* F, int S, int K, int M, const int* d2list,
                            int nrad, cx<double>* fk) {
  hipLaunchKernelGGL(k_polar_dft, dim3(nrad), dim3(256), 3 * (size_t)M * sizeof(double), s, F, S, K,
                     M, d2list, fk);
  return last();
}

hipError_t launch_synth_rotation(hipStream_t s, const float* F, int S, int K, const int* rmap,
                                 const cx<double>* fk, cx<double>* comps) {
  const int n = (K + 1) * S * S;
  hipLaunchKernelGGL(k_synth_rotation, dim3((n + 255) / 256), dim3(256), 0, s, F, S, K, rmap, fk,
                     comps);
  return last();
}

hipError_t launch_scale_components(hipStream_t s, double sigma0, double u_lo, double u_hi,
                                   double L, int n, int R, cx<double>* comps) {
  hipLaunchKernelGGL(k_scale_components, dim3(1), dim3(256), 0, s, sigma0, u_lo, u_hi, L, n, R,
                     comps);
  return last();
}

hipError_t launch_d2f(hipStream_t s, const cx<double>* in, cx<float>* out, long long n) {
  hipLaunchKernelGGL(k_d2f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
  return last();
}
hipError_t launch_conj_d(hipStream_t s, const cx<double>* in, cx<double>* out, long long n) {
  hipLaunchKernelGGL(k_conj_d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
  return last();
}
hipError_t launch_scale_f(hipStream_t s, float* y, long long n, float a) {
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_scale_f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, n, a);
  return last();
}
hipError_t launch_f2d(hipStream_t s, const cx<float>* in, cx<double>* out, long long n) {
  hipLaunchKernelGGL(k_f2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
  return last();
}

// Dynamic LDS above the default limit must be enabled per kernel.

hipError_t prepare_corr_kernels();
hipError_t prepare_conv_kernels();
hipError_t prepare_fixed_kernels();
hipError_t prepare_tile_kernels();
hipError_t prepare_tconv_kernels();

hipError_t prepare_kernels() {
  hipError_t e = prepare_corr_kernels();
  if (e == hipSuccess) e = prepare_conv_kernels();
  if (e == hipSuccess) e = prepare_fixed_kernels();
  if (e == hipSuccess) e = prepare_tile_kernels();
  if (e == hipSuccess) e = prepare_tconv_kernels();
  if (e == hipSuccess) e = prepare_fx_kernels();
#define ECC_ALLOW(...) if (e == hipSuccess) e = allow_lds(__VA_ARGS__)
#define ECC_ALLOW_NB(KN) ECC_ALLOW(KN<1>); ECC_ALLOW(KN<2>); ECC_ALLOW(KN<4>)
#define ECC_ALLOW_NB_E(KN, E) ECC_ALLOW(KN<1, E>); ECC_ALLOW(KN<2, E>); ECC_ALLOW(KN<4, E>)
#define ECC_ALLOW_EPX(KN) \
  ECC_ALLOW_NB_E(KN, 1); ECC_ALLOW_NB_E(KN, 2); ECC_ALLOW_NB_E(KN, 4); ECC_ALLOW_NB_E(KN, 8); ECC_ALLOW_NB_E(KN, 16)
#define ECC_ALLOW_GEN(T)                                                          \
  ECC_ALLOW(k_fft_rows<T, 1, -1>); ECC_ALLOW(k_fft_rows<T, 2, -1>); ECC_ALLOW(k_fft_rows<T, 4, -1>); \
  ECC_ALLOW(k_fft_rows<T, 1, 1>); ECC_ALLOW(k_fft_rows<T, 2, 1>); ECC_ALLOW(k_fft_rows<T, 4, 1>);    \
  ECC_ALLOW(k_fft_cols<T, 1, -1>); ECC_ALLOW(k_fft_cols<T, 2, -1>); ECC_ALLOW(k_fft_cols<T, 4, -1>); \
  ECC_ALLOW(k_fft_cols<T, 1, 1>); ECC_ALLOW(k_fft_cols<T, 2, 1>); ECC_ALLOW(k_fft_cols<T, 4, 1>)
  ECC_ALLOW_GEN(float);
  ECC_ALLOW_GEN(double);
  return e;
}

}  // namespace ecc
