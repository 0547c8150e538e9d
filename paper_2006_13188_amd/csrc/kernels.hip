// HIP kernels (gfx950) for spatially adaptive correlation and convolution by angular
// components (Sec. 4.1 of "Efficient Spatially Adaptive Convolution and Correlation").
//
// Correlation, for a real signal H and components F_k, k = 0..U-1:
//   rows_r2c   : A(i, v)   = FFT_x of H rows, half spectrum v in [0, W), W = Px/2 + 1
//   cols_fwd   : Hh(u, v)  = FFT_y of A columns (zero rows beyond ny)
//   corr_cols  : T_k(i, v) = IFFT_y(Hh conj Fh_k) cropped to i < ny, for all v in [0, Px);
//                the column Px - v comes from column v through conjugate symmetry of Hh
//   corr_rows  : y = scale * sum_k w_k Re(e^{i k alpha} IFFT_x(T_k)), cropped to nx
// Convolution (signal pre-multiplied by e^{-i k alpha}, Sec. 4.1):
//   conv_rows_fwd : B_k = FFT_x(H e^{-i k alpha})
//   conv_cols     : C = IFFT_y(sum_k w_k FFT_y(B_k) Fh_k), cropped to ny
//   conv_rows_inv : y = Re IFFT_x(C) (or the ratio of two such outputs)
// All global accesses are bounds-checked against the image, spectrum and plane sizes.
#include "kernels.hpp"

namespace ecc {

static __device__ __forceinline__ int lds_tw_pad(int n) { return (n + 1) & ~1; }

// ---------------------------------------------------------------------------------
// rows_r2c: two real rows packed as one complex transform, split after the FFT.
template <int NB>
__global__ void __launch_bounds__(256) k_rows_r2c(const float* __restrict__ H, long long planeH,
                                                 int ldH, cx<float>* __restrict__ A,
                                                 long long planeA, int ldA, int ny, int nx, int W,
                                                 FftDesc d, const cx<float>* __restrict__ tw,
                                                 int B, int TF) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int P = d.P;
  const int c = threadIdx.x / TF, f = threadIdx.x - c * TF;
  const int r0 = 2 * (blockIdx.x * B + c), r1 = r0 + 1;
  const bool active = (c < B) && (r0 < ny);
  const float* Hb = H + (long long)blockIdx.y * planeH;
  Layout L{B, 0, P};
  if (active) {
    for (int pos = f; pos < P; pos += TF) {
      float a = 0.f, b = 0.f;
      if (pos < nx) {
        a = Hb[(long long)r0 * ldH + pos];
        if (r1 < ny) b = Hb[(long long)r1 * ldH + pos];
      }
      buf[c * P + pos] = mk(a, b);
    }
  }
  __syncthreads();
  run_fft<NB, -1, false, float>(buf, L, d, twl, c, f, TF, active);
  if (active) {
    cx<float>* Ab = A + (long long)blockIdx.y * planeA;
    for (int v = f; v < W; v += TF) {
      const cx<float> z = buf[c * P + v];
      const cx<float> zm = buf[c * P + (v == 0 ? 0 : P - v)];
      Ab[(long long)r0 * ldA + v] = mk(0.5f * (z.re + zm.re), 0.5f * (z.im - zm.im));
      if (r1 < ny) Ab[(long long)r1 * ldA + v] = mk(0.5f * (z.im + zm.im), -0.5f * (z.re - zm.re));
    }
  }
}

// ---------------------------------------------------------------------------------
// cols_fwd: forward transform of B adjacent columns (rows >= nyValid are zero).
template <int NB>
__global__ void __launch_bounds__(512) k_cols_fwd(const cx<float>* __restrict__ A,
                                                 long long planeA, int ldA, int nyValid, int ncols,
                                                 cx<float>* __restrict__ out, long long planeOut,
                                                 int ldOut, FftDesc d,
                                                 const cx<float>* __restrict__ tw, int lgB) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int B = 1 << lgB, P = d.P, nthr = blockDim.x, TF = nthr >> lgB;
  const int c = threadIdx.x & (B - 1), f = threadIdx.x >> lgB;
  const int v0 = blockIdx.x * B;
  const cx<float>* Ab = A + (long long)blockIdx.y * planeA;
  for (int e = threadIdx.x; e < P * B; e += nthr) {
    const int pos = e >> lgB, v = v0 + (e & (B - 1));
    cx<float> val = mk(0.f, 0.f);
    if (pos < nyValid && v < ncols) val = Ab[(long long)pos * ldA + v];
    buf[e] = val;
  }
  __syncthreads();
  Layout L{B, lgB, 0};
  run_fft<NB, -1, true, float>(buf, L, d, twl, c, f, TF, true);
  cx<float>* Ob = out + (long long)blockIdx.y * planeOut;
  for (int e = threadIdx.x; e < P * B; e += nthr) {
    const int pos = e >> lgB, v = v0 + (e & (B - 1));
    if (v < ncols) Ob[(long long)pos * ldOut + v] = buf[e];
  }
}

// ---------------------------------------------------------------------------------
// corr_cols: per component, direct column v and mirror column Px - v. With
// a = F(u, v) and b = F(-u, -v) (read from a full-plane spectrum, or parity_k * a when
// the component satisfies F_k(-x) = parity_k F_k(x)):
//   conj_mode 0, G = IFFT(Hh conj F):     T(:, v) = IFFT(h conj a),  T(:, -v) = conj IFFT(h b)
//   conj_mode 1, G = IFFT(Hh F):          T(:, v) = IFFT(h a),       T(:, -v) = conj IFFT(h conj b)
//   conj_mode 2, G = IFFT(Hh(w) F(-w)):   T(:, v) = IFFT(h b),       T(:, -v) = conj IFFT(h conj a)
// (the mirror forms use Hh(u, -v) = conj Hh(-u, v) for a real signal and u -> -u).
template <int NB>
__global__ void __launch_bounds__(512) k_corr_cols(
    const cx<float>* __restrict__ Hh, long long planeHh, int ldHh, const cx<float>* __restrict__ Fh,
    long long planeFk, int ldF, int fullplane, const float* __restrict__ parity,
    cx<float>* __restrict__ T, long long planeTk, long long planeTimg, int ldT, int ny, int Px,
    int W, int U, int kchunk, int conj_mode, FftDesc d, const cx<float>* __restrict__ tw, int lgB) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int B = 1 << lgB, Py = d.P, nthr = blockDim.x, TF = nthr >> lgB;
  const int c = threadIdx.x & (B - 1), f = threadIdx.x >> lgB;
  const int v0 = blockIdx.x * B;
  const int k0 = blockIdx.y * kchunk;
  const int k1 = min(U, k0 + kchunk);
  const cx<float>* Hb = Hh + (long long)blockIdx.z * planeHh;
  Layout L{B, lgB, 0};
  for (int k = k0; k < k1; ++k) {
    const cx<float>* Fk = Fh + (long long)k * planeFk;
    cx<float>* Tk = T + (long long)blockIdx.z * planeTimg + (long long)k * planeTk;
    const float par = fullplane ? 1.f : parity[k];
    for (int half = 0; half < 2; ++half) {
      // which filter value (a or b) and whether it is conjugated
      const bool use_b = (conj_mode == 0) ? (half == 1) : (conj_mode == 1 ? (half == 1) : (half == 0));
      const bool use_conj = (conj_mode == 0) ? (half == 0) : (half == 1);
      for (int e = threadIdx.x; e < Py * B; e += nthr) {
        const int u = e >> lgB, v = v0 + (e & (B - 1));
        cx<float> val = mk(0.f, 0.f);
        if (v < W) {
          const cx<float> h = Hb[(long long)u * ldHh + v];
          cx<float> g;
          if (!use_b) {
            g = Fk[(long long)u * ldF + v];
          } else if (!fullplane) {
            g = scale(Fk[(long long)u * ldF + v], par);
          } else {
            const int um = (u == 0) ? 0 : Py - u;
            const int vm = (v == 0) ? 0 : Px - v;
            g = Fk[(long long)um * ldF + vm];
          }
          val = use_conj ? cmulc(h, g) : cmul(h, g);
        }
        buf[e] = val;
      }
      __syncthreads();
      run_fft<NB, +1, true, float>(buf, L, d, twl, c, f, TF, true);
      for (int e = threadIdx.x; e < ny * B; e += nthr) {
        const int i = e >> lgB, v = v0 + (e & (B - 1));
        if (v >= W) continue;
        const cx<float> r = buf[e];
        if (half == 0) {
          Tk[(long long)i * ldT + v] = r;
        } else if (v != 0 && 2 * v != Px) {
          Tk[(long long)i * ldT + (Px - v)] = conj(r);
        }
      }
      // the next product overwrites only this thread's own elements (same e mapping)
    }
  }
}

// ---------------------------------------------------------------------------------
// per-pixel phase helpers (float64 recurrence, rounded when used)
struct Phase {
  double re, im;
};
__device__ __forceinline__ Phase pmul(Phase a, Phase b) {
  Phase r;
  r.re = a.re * b.re - a.im * b.im;
  r.im = a.re * b.im + a.im * b.re;
  return r;
}
__device__ __forceinline__ double field_angle(const Field& f, float v) {
  const double x = f.log_mode ? log((double)v) : (double)v;
  return f.mul * x + f.add;
}

// corr_rows: inverse row transforms of every component and the per-pixel combination.
// Optional second output y2 = y2scale * mulsig * sum_k w_k k Im(e^{ik alpha} G_k) (adjoint).
template <int NB, int EPX>
__global__ void __launch_bounds__(256) k_corr_rows(
    const cx<float>* __restrict__ T, long long planeTk, long long planeTimg, int ldT, Field fld,
    float* __restrict__ y, long long planeY, int ldY, int ny, int nx, int U,
    const float* __restrict__ w, float scl, float* __restrict__ y2,
    const float* __restrict__ mulsig, long long planeMul, int ldMul, float y2scale, FftDesc d,
    const cx<float>* __restrict__ tw, int B, int TF) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int Px = d.P;
  const int c = threadIdx.x / TF, f = threadIdx.x - c * TF;
  const int row = blockIdx.x * B + c;
  const bool active = (c < B) && (row < ny);
  const int img = blockIdx.y;
  Layout L{B, 0, Px};
  Phase z[EPX], e1[EPX];
  float acc[EPX], acc2[EPX];
#pragma unroll
  for (int j = 0; j < EPX; ++j) {
    const int x = f + j * TF;
    z[j].re = 1.0;
    z[j].im = 0.0;
    e1[j] = z[j];
    acc[j] = 0.f;
    acc2[j] = 0.f;
    if (active && x < nx) {
      const double a = field_angle(fld, fld.ptr[(long long)img * fld.plane + (long long)row * fld.ld + x]);
      double sn, cs;
      sincos(a, &sn, &cs);
      e1[j].re = cs;
      e1[j].im = sn;
    }
  }
  const cx<float>* Tb = T + (long long)img * planeTimg + (long long)row * ldT;
  for (int k = 0; k < U; ++k) {
    if (active) {
      const cx<float>* src = Tb + (long long)k * planeTk;
      for (int pos = f; pos < Px; pos += TF) buf[c * Px + pos] = src[pos];
    }
    __syncthreads();
    run_fft<NB, +1, false, float>(buf, L, d, twl, c, f, TF, active);
    const float wk = w[k];
#pragma unroll
    for (int j = 0; j < EPX; ++j) {
      const int x = f + j * TF;
      if (active && x < nx) {
        const cx<float> g = buf[c * Px + x];
        const float zr = (float)z[j].re, zi = (float)z[j].im;
        acc[j] += wk * (zr * g.re - zi * g.im);
        if (y2) acc2[j] += wk * (float)k * (zr * g.im + zi * g.re);
      }
      z[j] = pmul(z[j], e1[j]);
    }
  }
  if (active) {
#pragma unroll
    for (int j = 0; j < EPX; ++j) {
      const int x = f + j * TF;
      if (x < nx) {
        y[(long long)img * planeY + (long long)row * ldY + x] = acc[j] * scl;
        if (y2)
          y2[(long long)img * planeY + (long long)row * ldY + x] =
              acc2[j] * scl * y2scale * mulsig[(long long)img * planeMul + (long long)row * ldMul + x];
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// match_rows: response at n_angles equispaced angles, C(m) = sum_k w_k Re(e^{2 pi i k m / A} G_k),
// kept per pixel in registers; best score and the smallest maximising index.
template <int NB, int EPX>
__global__ void __launch_bounds__(512) k_match_rows(
    const cx<float>* __restrict__ T, long long planeTk, int ldT, float* __restrict__ score,
    int* __restrict__ index, int ldOut, int ny, int nx, int U, const float* __restrict__ w,
    float scl, int A, const float* __restrict__ angle_tab, FftDesc d,
    const cx<float>* __restrict__ tw, int B, int TF) {
  constexpr int AMAX = 64;
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  float* ctab = (float*)(smem_f + lds_tw_pad(d.twsize));   // cos(2 pi t / A), t < A
  float* stab = ctab + AMAX;                               // sin(2 pi t / A)
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize) + AMAX;   // 2*AMAX floats = AMAX complex
  for (int i = threadIdx.x; i < A; i += blockDim.x) {
    ctab[i] = angle_tab[i];
    stab[i] = angle_tab[AMAX + i];
  }
  stage_twiddles(twl, tw, d.twsize);
  const int Px = d.P;
  const int c = threadIdx.x / TF, f = threadIdx.x - c * TF;
  const int row = blockIdx.x * B + c;
  const bool active = (c < B) && (row < ny);
  Layout L{B, 0, Px};
  float acc[EPX][AMAX];
#pragma unroll
  for (int j = 0; j < EPX; ++j)
#pragma unroll
    for (int m = 0; m < AMAX; ++m) acc[j][m] = 0.f;
  const cx<float>* Tb = T + (long long)row * ldT;
  for (int k = 0; k < U; ++k) {
    if (active) {
      const cx<float>* src = Tb + (long long)k * planeTk;
      for (int pos = f; pos < Px; pos += TF) buf[c * Px + pos] = src[pos];
    }
    __syncthreads();
    run_fft<NB, +1, false, float>(buf, L, d, twl, c, f, TF, active);
    const float wk = w[k];
#pragma unroll
    for (int j = 0; j < EPX; ++j) {
      const int x = f + j * TF;
      if (active && x < nx) {
        const cx<float> g = buf[c * Px + x];
        const float gr = wk * g.re, gi = wk * g.im;
        int t = 0;
#pragma unroll
        for (int m = 0; m < AMAX; ++m) {
          if (m < A) {
            acc[j][m] += gr * ctab[t] - gi * stab[t];
            t += k;   // k < A because A >= 2K + 1
            if (t >= A) t -= A;
          }
        }
      }
    }
  }
  if (active) {
#pragma unroll
    for (int j = 0; j < EPX; ++j) {
      const int x = f + j * TF;
      if (x < nx) {
        float best = acc[j][0];
        int bi = 0;
#pragma unroll
        for (int m = 1; m < AMAX; ++m)
          if (m < A && acc[j][m] > best) {
            best = acc[j][m];
            bi = m;
          }
        score[(long long)row * ldOut + x] = best * scl;
        index[(long long)row * ldOut + x] = bi;
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// conv_rows_fwd: B_{k,s} = FFT_x(sig_s e^{-i k alpha}); sig_0 = H (or H / s^2 when
// sig_norm), sig_1 = 1 / s^2 (the constant signal of the normalising denominator).
template <int NB, int EPX>
__global__ void __launch_bounds__(256) k_conv_rows_fwd(
    const float* __restrict__ H, long long planeH, int ldH, Field fld, int sig_norm, int nsig,
    cx<float>* __restrict__ Bk, long long planeBk, long long planeBsig, long long planeBimg, int ldB,
    int ny, int nx, int U, FftDesc d, const cx<float>* __restrict__ tw, int B, int TF) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int Px = d.P;
  const int c = threadIdx.x / TF, f = threadIdx.x - c * TF;
  const int row = blockIdx.x * B + c;
  const bool active = (c < B) && (row < ny);
  const int img = blockIdx.y;
  Layout L{B, 0, Px};
  Phase z[EPX], e1[EPX];
  double sg[2][EPX];
#pragma unroll
  for (int j = 0; j < EPX; ++j) {
    const int x = f + j * TF;
    z[j].re = 1.0;
    z[j].im = 0.0;
    e1[j] = z[j];
    sg[0][j] = 0.0;
    sg[1][j] = 0.0;
    if (active && x < nx) {
      const float fv = fld.ptr[(long long)img * fld.plane + (long long)row * fld.ld + x];
      const double a = field_angle(fld, fv);
      double sn, cs;
      sincos(a, &sn, &cs);
      e1[j].re = cs;
      e1[j].im = -sn;   // e^{-i alpha}
      const double h = (double)H[(long long)img * planeH + (long long)row * ldH + x];
      const double wn = sig_norm ? 1.0 / ((double)fv * (double)fv) : 1.0;
      sg[0][j] = h * wn;
      sg[1][j] = wn;
    }
  }
  for (int k = 0; k < U; ++k) {
    for (int s = 0; s < nsig; ++s) {
      if (active) {
        for (int pos = nx + f; pos < Px; pos += TF) buf[c * Px + pos] = mk(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < EPX; ++j) {
          const int x = f + j * TF;
          if (x < nx) buf[c * Px + x] = mk((float)(sg[s][j] * z[j].re), (float)(sg[s][j] * z[j].im));
        }
      }
      __syncthreads();
      run_fft<NB, -1, false, float>(buf, L, d, twl, c, f, TF, active);
      if (active) {
        cx<float>* dst = Bk + (long long)img * planeBimg + (long long)s * planeBsig +
                         (long long)k * planeBk + (long long)row * ldB;
        for (int pos = f; pos < Px; pos += TF) dst[pos] = buf[c * Px + pos];
      }
      __syncthreads();   // the next signal overwrites positions other threads just stored
    }
#pragma unroll
    for (int j = 0; j < EPX; ++j) z[j] = pmul(z[j], e1[j]);
  }
}

// ---------------------------------------------------------------------------------
// conv_cols: forward column transforms of every B_k, products with the filter spectra,
// accumulation over k in registers, one inverse column transform, crop to ny rows.
// F(u, v) for v >= W comes from F(-u, -v) (full plane) or parity_k * F(Py-u, Px-v).
template <int NB, int EPT>
__global__ void __launch_bounds__(512) k_conv_cols(
    const cx<float>* __restrict__ Bk, long long planeBk, long long planeBsig, long long planeBimg,
    int ldB, const cx<float>* __restrict__ Fh, long long planeFk, int ldF, int fullplane,
    const float* __restrict__ parity, const float* __restrict__ w, cx<float>* __restrict__ C,
    long long planeCsig, long long planeCimg, int ldC, int ny, int Px, int W, int U, int nsig,
    FftDesc d, const cx<float>* __restrict__ tw, int lgB) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int B = 1 << lgB, Py = d.P, nthr = blockDim.x, TF = nthr >> lgB;
  const int c = threadIdx.x & (B - 1), f = threadIdx.x >> lgB;
  const int v0 = blockIdx.x * B;
  const int img = blockIdx.y;
  Layout L{B, lgB, 0};
  cx<float> Z[2][EPT];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int j = 0; j < EPT; ++j) Z[s][j] = mk(0.f, 0.f);
  for (int k = 0; k < U; ++k) {
    const cx<float>* Fk = Fh + (long long)k * planeFk;
    const float wk = w[k];
    const float par = fullplane ? 1.f : parity[k];
    for (int s = 0; s < nsig; ++s) {
      const cx<float>* src = Bk + (long long)img * planeBimg + (long long)s * planeBsig + (long long)k * planeBk;
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int e = threadIdx.x + j * nthr;
        if (e < Py * B) {
          const int i = e >> lgB, v = v0 + (e & (B - 1));
          cx<float> val = mk(0.f, 0.f);
          if (i < ny && v < Px) val = src[(long long)i * ldB + v];
          buf[e] = val;
        }
      }
      __syncthreads();
      run_fft<NB, -1, true, float>(buf, L, d, twl, c, f, TF, true);
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int e = threadIdx.x + j * nthr;
        if (e < Py * B) {
          const int u = e >> lgB, v = v0 + (e & (B - 1));
          if (v < Px) {
            cx<float> g;
            if (fullplane || v < W) {
              g = Fk[(long long)u * ldF + v];
            } else {
              const int um = (u == 0) ? 0 : Py - u;
              g = scale(Fk[(long long)um * ldF + (Px - v)], par);
            }
            const cx<float> p = cmul(buf[e], g);
            Z[s][j].re += wk * p.re;
            Z[s][j].im += wk * p.im;
          }
        }
      }
    }
  }
  for (int s = 0; s < nsig; ++s) {
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = threadIdx.x + j * nthr;
      if (e < Py * B) buf[e] = Z[s][j];
    }
    __syncthreads();
    run_fft<NB, +1, true, float>(buf, L, d, twl, c, f, TF, true);
    cx<float>* dst = C + (long long)img * planeCimg + (long long)s * planeCsig;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = threadIdx.x + j * nthr;
      if (e < ny * B) {
        const int i = e >> lgB, v = v0 + (e & (B - 1));
        if (v < Px) dst[(long long)i * ldC + v] = buf[e];
      }
    }
  }
}

// conv_rows_inv: y = scale * Re IFFT_x(C_0), or Re IFFT_x(C_0) / Re IFFT_x(C_1).
template <int NB, int EPX>
__global__ void __launch_bounds__(256) k_conv_rows_inv(
    const cx<float>* __restrict__ C, long long planeCsig, long long planeCimg, int ldC,
    float* __restrict__ y, long long planeY, int ldY, int ny, int nx, int nsig, float scl,
    FftDesc d, const cx<float>* __restrict__ tw, int B, int TF) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int Px = d.P;
  const int c = threadIdx.x / TF, f = threadIdx.x - c * TF;
  const int row = blockIdx.x * B + c;
  const bool active = (c < B) && (row < ny);
  const int img = blockIdx.y;
  Layout L{B, 0, Px};
  float r[2][EPX];
  for (int s = 0; s < nsig; ++s) {
    if (active) {
      const cx<float>* src = C + (long long)img * planeCimg + (long long)s * planeCsig + (long long)row * ldC;
      for (int pos = f; pos < Px; pos += TF) buf[c * Px + pos] = src[pos];
    }
    __syncthreads();
    run_fft<NB, +1, false, float>(buf, L, d, twl, c, f, TF, active);
#pragma unroll
    for (int j = 0; j < EPX; ++j) {
      const int x = f + j * TF;
      r[s][j] = (active && x < nx) ? buf[c * Px + x].re : 0.f;
    }
  }
  if (active) {
#pragma unroll
    for (int j = 0; j < EPX; ++j) {
      const int x = f + j * TF;
      if (x < nx) {
        const float v = (nsig == 2) ? r[0][j] / r[1][j] : r[0][j] * scl;
        y[(long long)img * planeY + (long long)row * ldY + x] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// generic complex transforms with circular placement:
//   rows: buf[(j + shift_in) mod P] = in[r][j] for j < nvalid; out[r][i] = buf[(i + shift_out) mod P]
//   cols: the same along columns of B adjacent columns.
template <typename T, int NB, int DIR>
__global__ void __launch_bounds__(256) k_fft_rows(const cx<T>* __restrict__ in, long long planeIn,
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
    for (int pos = f; pos < P; pos += TF) {
      int j = pos - shift_in;
      j %= P;
      if (j < 0) j += P;
      cx<T> val;
      val.re = T(0);
      val.im = T(0);
      if (j < nvalid) val = src[j];
      buf[c * P + pos] = val;
    }
  }
  __syncthreads();
  run_fft<NB, DIR, false, T>(buf, L, d, twl, c, f, TF, active);
  if (active) {
    cx<T>* dst = out + (long long)blockIdx.y * planeOut + (long long)row * ldOut;
    for (int i = f; i < nstore; i += TF) {
      int pos = (i + shift_out) % P;
      if (pos < 0) pos += P;
      dst[i] = buf[c * P + pos];
    }
  }
}

template <typename T, int NB, int DIR>
__global__ void __launch_bounds__(512) k_fft_cols(const cx<T>* __restrict__ in, long long planeIn,
                                                 int ldIn, int ncols, int nvalid, int shift_in,
                                                 cx<T>* __restrict__ out, long long planeOut,
                                                 int ldOut, int nstore, int shift_out, FftDesc d,
                                                 const cx<T>* __restrict__ tw, int lgB) {
  extern __shared__ char smem_raw[];
  cx<T>* twl = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = twl + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int B = 1 << lgB, P = d.P, nthr = blockDim.x, TF = nthr >> lgB;
  const int c = threadIdx.x & (B - 1), f = threadIdx.x >> lgB;
  const int v0 = blockIdx.x * B;
  const cx<T>* src = in + (long long)blockIdx.y * planeIn;
  for (int e = threadIdx.x; e < P * B; e += nthr) {
    const int pos = e >> lgB, v = v0 + (e & (B - 1));
    int j = (pos - shift_in) % P;
    if (j < 0) j += P;
    cx<T> val;
    val.re = T(0);
    val.im = T(0);
    if (j < nvalid && v < ncols) val = src[(long long)j * ldIn + v];
    buf[e] = val;
  }
  __syncthreads();
  Layout L{B, lgB, 0};
  run_fft<NB, DIR, true, T>(buf, L, d, twl, c, f, TF, true);
  cx<T>* dst = out + (long long)blockIdx.y * planeOut;
  for (int e = threadIdx.x; e < nstore * B; e += nthr) {
    const int i = e >> lgB, v = v0 + (e & (B - 1));
    if (v >= ncols) continue;
    int pos = (i + shift_out) % P;
    if (pos < 0) pos += P;
    dst[(long long)i * ldOut + v] = buf[(pos << lgB) + (e & (B - 1))];
  }
}

// ---------------------------------------------------------------------------------
// adjoint of the convolution w.r.t. the components: D_k(u, v) = sum_b Gh_b(u, v) conj(FFT_y(B_{k,b})(u, v))
// (fixed batch order, no atomics).
template <int NB>
__global__ void __launch_bounds__(512) k_grad_filter_cols(
    const cx<float>* __restrict__ Bk, long long planeBk, long long planeBimg, int ldB,
    const cx<float>* __restrict__ Gh, long long planeGimg, int ldG, cx<float>* __restrict__ D,
    long long planeDk, int ldD, int ny, int Px, int W, int batch, FftDesc d,
    const cx<float>* __restrict__ tw, int lgB) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int B = 1 << lgB, Py = d.P, nthr = blockDim.x, TF = nthr >> lgB;
  const int c = threadIdx.x & (B - 1), f = threadIdx.x >> lgB;
  const int v0 = blockIdx.x * B;
  const int k = blockIdx.y;
  Layout L{B, lgB, 0};
  cx<float>* Dk = D + (long long)k * planeDk;
  for (int b = 0; b < batch; ++b) {
    const cx<float>* src = Bk + (long long)b * planeBimg + (long long)k * planeBk;
    for (int e = threadIdx.x; e < Py * B; e += nthr) {
      const int i = e >> lgB, v = v0 + (e & (B - 1));
      cx<float> val = mk(0.f, 0.f);
      if (i < ny && v < Px) val = src[(long long)i * ldB + v];
      buf[e] = val;
    }
    __syncthreads();
    run_fft<NB, -1, true, float>(buf, L, d, twl, c, f, TF, true);
    const cx<float>* G = Gh + (long long)b * planeGimg;
    for (int e = threadIdx.x; e < Py * B; e += nthr) {
      const int u = e >> lgB, v = v0 + (e & (B - 1));
      if (v < Px) {
        // Gh holds columns [0, W) of the spectrum of a real image; the rest by symmetry
        cx<float> gv;
        if (v < W) {
          gv = G[(long long)u * ldG + v];
        } else {
          const int um = (u == 0) ? 0 : Py - u;
          gv = conj(G[(long long)um * ldG + (Px - v)]);
        }
        const cx<float> p = cmulc(gv, buf[e]);
        cx<float>* dst = Dk + (long long)u * ldD + v;
        if (b == 0) *dst = p;
        else *dst = *dst + p;
      }
    }
    __syncthreads();
  }
}

__global__ void k_grad_filter_finish(const cx<float>* __restrict__ win, long long planeWin,
                                     int ldWin, const float* __restrict__ w, float scl,
                                     cx<float>* __restrict__ out, int S, int U) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= U * S * S) return;
  const int k = idx / (S * S), rem = idx - k * S * S;
  const int a = rem / S, b = rem - a * S;
  const cx<float> v = win[(long long)k * planeWin + (long long)a * ldWin + b];
  out[idx] = scale(v, w[k] * scl);
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
size_t lds_rows(const RowCfg& c, const FftDesc& d, size_t elem) {
  return elem * ((size_t)((d.twsize + 1) & ~1) + (size_t)c.B * d.P);
}
size_t lds_cols(const ColCfg& c, const FftDesc& d, size_t elem) {
  return elem * ((size_t)((d.twsize + 1) & ~1) + ((size_t)d.P << c.lgB));
}

#define ECC_NB_SWITCH(NBV, ...)                         \
  switch (NBV) {                                        \
    case 1: { constexpr int NB = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int NB = 2; __VA_ARGS__; } break; \
    case 4: { constexpr int NB = 4; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;               \
  }
#define ECC_EPX_SWITCH(EV, ...)                          \
  switch (EV) {                                          \
    case 1: { constexpr int EPX = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int EPX = 2; __VA_ARGS__; } break; \
    case 4: { constexpr int EPX = 4; __VA_ARGS__; } break; \
    case 8: { constexpr int EPX = 8; __VA_ARGS__; } break; \
    case 16: { constexpr int EPX = 16; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                \
  }
#define ECC_EPT_SWITCH(EV, ...)                          \
  switch (EV) {                                          \
    case 4: { constexpr int EPT = 4; __VA_ARGS__; } break; \
    case 8: { constexpr int EPT = 8; __VA_ARGS__; } break; \
    case 12: { constexpr int EPT = 12; __VA_ARGS__; } break; \
    case 16: { constexpr int EPT = 16; __VA_ARGS__; } break; \
    case 24: { constexpr int EPT = 24; __VA_ARGS__; } break; \
    case 32: { constexpr int EPT = 32; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                \
  }

static inline hipError_t last() { return hipGetLastError(); }

hipError_t launch_rows_r2c(hipStream_t s, const RowCfg& c, int batch, const float* H, long long planeH,
                           int ldH, cx<float>* A, long long planeA, int ldA, int ny, int nx, int W,
                           const FftDesc& d, const cx<float>* tw) {
  const int pairs = (ny + 1) / 2;
  dim3 grid((pairs + c.B - 1) / c.B, batch), block(c.B * c.TF);
  const size_t lds = lds_rows(c, d, sizeof(cx<float>));
  ECC_NB_SWITCH(c.NB, hipLaunchKernelGGL(k_rows_r2c<NB>, grid, block, lds, s, H, planeH, ldH, A,
                                         planeA, ldA, ny, nx, W, d, tw, c.B, c.TF));
  return last();
}

hipError_t launch_cols_fwd(hipStream_t s, const ColCfg& c, int batch, const cx<float>* A,
                           long long planeA, int ldA, int nyValid, int ncols, cx<float>* out,
                           long long planeOut, int ldOut, const FftDesc& d, const cx<float>* tw) {
  const int B = 1 << c.lgB;
  dim3 grid((ncols + B - 1) / B, batch), block(c.nthr);
  const size_t lds = lds_cols(c, d, sizeof(cx<float>));
  ECC_NB_SWITCH(c.NB, hipLaunchKernelGGL(k_cols_fwd<NB>, grid, block, lds, s, A, planeA, ldA,
                                         nyValid, ncols, out, planeOut, ldOut, d, tw, c.lgB));
  return last();
}

hipError_t launch_corr_cols(hipStream_t s, const ColCfg& c, int batch, int kchunk,
                            const cx<float>* Hh, long long planeHh, int ldHh, const cx<float>* Fh,
                            long long planeFk, int ldF, int fullplane, const float* parity,
                            cx<float>* T, long long planeTk, long long planeTimg, int ldT, int ny,
                            int Px, int W, int U, int conj_mode, const FftDesc& d,
                            const cx<float>* tw) {
  const int B = 1 << c.lgB;
  dim3 grid((W + B - 1) / B, (U + kchunk - 1) / kchunk, batch), block(c.nthr);
  const size_t lds = lds_cols(c, d, sizeof(cx<float>));
  ECC_NB_SWITCH(c.NB, hipLaunchKernelGGL(k_corr_cols<NB>, grid, block, lds, s, Hh, planeHh, ldHh,
                                         Fh, planeFk, ldF, fullplane, parity, T, planeTk, planeTimg,
                                         ldT, ny, Px, W, U, kchunk, conj_mode, d, tw, c.lgB));
  return last();
}

hipError_t launch_corr_rows(hipStream_t s, const RowCfg& c, int batch, const cx<float>* T,
                            long long planeTk, long long planeTimg, int ldT, const Field& fld,
                            float* y, long long planeY, int ldY, int ny, int nx, int U,
                            const float* w, float scale_, float* y2, const float* mulsig,
                            long long planeMul, int ldMul, float y2scale, const FftDesc& d,
                            const cx<float>* tw) {
  dim3 grid((ny + c.B - 1) / c.B, batch), block(c.B * c.TF);
  const size_t lds = lds_rows(c, d, sizeof(cx<float>));
  ECC_NB_SWITCH(c.NB, ECC_EPX_SWITCH(c.EPX, hipLaunchKernelGGL((k_corr_rows<NB, EPX>), grid, block, lds, s,
                                         T, planeTk, planeTimg, ldT, fld, y, planeY, ldY, ny, nx, U,
                                         w, scale_, y2, mulsig, planeMul, ldMul, y2scale, d, tw, c.B,
                                         c.TF)));
  return last();
}

hipError_t launch_match_rows(hipStream_t s, const RowCfg& c, const cx<float>* T, long long planeTk,
                             int ldT, float* score, int* index, int ldOut, int ny, int nx, int U,
                             const float* w, float scale_, int n_angles, const float* angle_tab,
                             const FftDesc& d, const cx<float>* tw) {
  dim3 grid((ny + c.B - 1) / c.B), block(c.B * c.TF);
  const size_t lds = lds_rows(c, d, sizeof(cx<float>)) + 64 * sizeof(cx<float>);
  ECC_NB_SWITCH(c.NB, ECC_EPX_SWITCH(c.EPX, hipLaunchKernelGGL((k_match_rows<NB, EPX>), grid, block, lds, s,
                                         T, planeTk, ldT, score, index, ldOut, ny, nx, U, w, scale_,
                                         n_angles, angle_tab, d, tw, c.B, c.TF)));
  return last();
}

hipError_t launch_conv_rows_fwd(hipStream_t s, const RowCfg& c, int batch, const float* H,
                                long long planeH, int ldH, const Field& fld, int sig_norm,
                                int nsig, cx<float>* Bk, long long planeBk, long long planeBsig,
                                long long planeBimg, int ldB, int ny, int nx, int U,
                                const FftDesc& d, const cx<float>* tw) {
  dim3 grid((ny + c.B - 1) / c.B, batch), block(c.B * c.TF);
  const size_t lds = lds_rows(c, d, sizeof(cx<float>));
  ECC_NB_SWITCH(c.NB, ECC_EPX_SWITCH(c.EPX, hipLaunchKernelGGL((k_conv_rows_fwd<NB, EPX>), grid, block, lds, s,
                                         H, planeH, ldH, fld, sig_norm, nsig, Bk, planeBk,
                                         planeBsig, planeBimg, ldB, ny, nx, U, d, tw, c.B, c.TF)));
  return last();
}

hipError_t launch_conv_cols(hipStream_t s, const ColCfg& c, int batch, const cx<float>* Bk,
                            long long planeBk, long long planeBsig, long long planeBimg, int ldB,
                            const cx<float>* Fh, long long planeFk, int ldF, int fullplane,
                            const float* parity, const float* w, cx<float>* C, long long planeCsig,
                            long long planeCimg, int ldC, int ny, int Py, int Px, int W, int U,
                            int nsig, const FftDesc& d, const cx<float>* tw) {
  (void)Py;
  const int B = 1 << c.lgB;
  dim3 grid((Px + B - 1) / B, batch), block(c.nthr);
  const size_t lds = lds_cols(c, d, sizeof(cx<float>));
  ECC_NB_SWITCH(c.NB, ECC_EPT_SWITCH(c.EPT, hipLaunchKernelGGL((k_conv_cols<NB, EPT>), grid, block, lds, s,
                                         Bk, planeBk, planeBsig, planeBimg, ldB, Fh, planeFk, ldF,
                                         fullplane, parity, w, C, planeCsig, planeCimg, ldC, ny, Px,
                                         W, U, nsig, d, tw, c.lgB)));
  return last();
}

hipError_t launch_conv_rows_inv(hipStream_t s, const RowCfg& c, int batch, const cx<float>* C,
                                long long planeCsig, long long planeCimg, int ldC, float* y,
                                long long planeY, int ldY, int ny, int nx, int nsig, float scale_,
                                const FftDesc& d, const cx<float>* tw) {
  dim3 grid((ny + c.B - 1) / c.B, batch), block(c.B * c.TF);
  const size_t lds = lds_rows(c, d, sizeof(cx<float>));
  ECC_NB_SWITCH(c.NB, ECC_EPX_SWITCH(c.EPX, hipLaunchKernelGGL((k_conv_rows_inv<NB, EPX>), grid, block, lds, s,
                                         C, planeCsig, planeCimg, ldC, y, planeY, ldY, ny, nx, nsig,
                                         scale_, d, tw, c.B, c.TF)));
  return last();
}

template <typename T>
hipError_t launch_fft_rows(hipStream_t s, const RowCfg& c, int nplanes, int dir, const cx<T>* in,
                           long long planeIn, int ldIn, int nrows, int nvalid, int shift_in,
                           cx<T>* out, long long planeOut, int ldOut, int nstore, int shift_out,
                           const FftDesc& d, const cx<T>* tw) {
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
                           const FftDesc& d, const cx<T>* tw) {
  const int B = 1 << c.lgB;
  dim3 grid((ncols + B - 1) / B, nplanes), block(c.nthr);
  const size_t lds = lds_cols(c, d, sizeof(cx<T>));
  if (dir < 0) {
    ECC_NB_SWITCH(c.NB, hipLaunchKernelGGL((k_fft_cols<T, NB, -1>), grid, block, lds, s, in, planeIn,
                                           ldIn, ncols, nvalid, shift_in, out, planeOut, ldOut,
                                           nstore, shift_out, d, tw, c.lgB));
  } else {
    ECC_NB_SWITCH(c.NB, hipLaunchKernelGGL((k_fft_cols<T, NB, +1>), grid, block, lds, s, in, planeIn,
                                           ldIn, ncols, nvalid, shift_in, out, planeOut, ldOut,
                                           nstore, shift_out, d, tw, c.lgB));
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
                                           int, int, const FftDesc&, const cx<float>*);
template hipError_t launch_fft_cols<double>(hipStream_t, const ColCfg&, int, int, const cx<double>*,
                                            long long, int, int, int, int, cx<double>*, long long,
                                            int, int, int, const FftDesc&, const cx<double>*);

hipError_t launch_grad_filter_cols(hipStream_t s, const ColCfg& c, int batch,
                                   const cx<float>* Bk, long long planeBk, long long planeBimg,
                                   int ldB, const cx<float>* Gh, long long planeGimg, int ldG,
                                   cx<float>* D, long long planeDk, int ldD, int ny, int Py, int Px,
                                   int U, const FftDesc& d, const cx<float>* tw) {
  (void)Py;
  const int B = 1 << c.lgB;
  dim3 grid((Px + B - 1) / B, U), block(c.nthr);
  const size_t lds = lds_cols(c, d, sizeof(cx<float>));
  ECC_NB_SWITCH(c.NB, hipLaunchKernelGGL(k_grad_filter_cols<NB>, grid, block, lds, s, Bk, planeBk,
                                         planeBimg, ldB, Gh, planeGimg, ldG, D, planeDk, ldD, ny,
                                         Px, Px / 2 + 1, batch, d, tw, c.lgB));
  return last();
}

hipError_t launch_grad_filter_finish(hipStream_t s, const cx<float>* win, long long planeWin,
                                     int ldWin, const float* w, float scale_, cx<float>* out, int S,
                                     int U) {
  const int n = U * S * S;
  hipLaunchKernelGGL(k_grad_filter_finish, dim3((n + 255) / 256), dim3(256), 0, s, win, planeWin,
                     ldWin, w, scale_, out, S, U);
  return last();
}

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
hipError_t launch_f2d(hipStream_t s, const cx<float>* in, cx<double>* out, long long n) {
  hipLaunchKernelGGL(k_f2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
  return last();
}

// Dynamic LDS above the default limit must be enabled per kernel.
template <typename K>
static hipError_t allow_lds(K kernel) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

hipError_t prepare_kernels() {
  hipError_t e = hipSuccess;
#define ECC_ALLOW(...) if (e == hipSuccess) e = allow_lds(__VA_ARGS__)
#define ECC_ALLOW_NB(KN)                                      \
  ECC_ALLOW(KN<1>);                                           \
  ECC_ALLOW(KN<2>);                                           \
  ECC_ALLOW(KN<4>)
  ECC_ALLOW_NB(k_rows_r2c);
  ECC_ALLOW_NB(k_cols_fwd);
  ECC_ALLOW_NB(k_corr_cols);
  ECC_ALLOW_NB(k_grad_filter_cols);
#define ECC_ALLOW_NB_E(KN, E) ECC_ALLOW(KN<1, E>); ECC_ALLOW(KN<2, E>); ECC_ALLOW(KN<4, E>)
#define ECC_ALLOW_EPX(KN) \
  ECC_ALLOW_NB_E(KN, 1); ECC_ALLOW_NB_E(KN, 2); ECC_ALLOW_NB_E(KN, 4); ECC_ALLOW_NB_E(KN, 8); ECC_ALLOW_NB_E(KN, 16)
  ECC_ALLOW_EPX(k_corr_rows);
  ECC_ALLOW_EPX(k_match_rows);
  ECC_ALLOW_EPX(k_conv_rows_fwd);
  ECC_ALLOW_EPX(k_conv_rows_inv);
  ECC_ALLOW_NB_E(k_conv_cols, 4); ECC_ALLOW_NB_E(k_conv_cols, 8); ECC_ALLOW_NB_E(k_conv_cols, 12);
  ECC_ALLOW_NB_E(k_conv_cols, 16); ECC_ALLOW_NB_E(k_conv_cols, 24); ECC_ALLOW_NB_E(k_conv_cols, 32);
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
