// HIP kernels (gfx950) of the extended-convolution path (Sec. 4.1: the signal is
// multiplied by e^{-i k alpha} before the k-th convolution) and of its adjoint:
//   conv_rows_fwd : B_k = FFT_x(H e^{-i k alpha})
//   conv_cols     : C = IFFT_y(sum_k w_k FFT_y(B_k) Fh_k), cropped to ny
//   conv_rows_inv : y = Re IFFT_x(C) (or the ratio of two such outputs)
//   grad_filter_* : gradient with respect to the components
// All global accesses are bounds-checked against the image, spectrum and plane sizes.
#include "kcommon.hpp"

namespace ecc {

// ---------------------------------------------------------------------------------
// conv_rows_fwd: B_{k,s} = FFT_x(sig_s e^{-i k alpha}); sig_0 = H (or H / s^2 when
// sig_norm), sig_1 = 1 / s^2 (the constant signal of the normalising denominator).
template <int NB, int EPX>
__global__ void __launch_bounds__(512) k_conv_rows_fwd(
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
    FftDesc d, const cx<float>* __restrict__ tw, int lgB, int per, cx<float>* __restrict__ part) {
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
  // component group blockIdx.z: components [k0, k1)
  const int k0 = blockIdx.z * per, k1 = min(U, k0 + per);
  for (int k = k0; k < k1; ++k) {
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
  if (part) {
    // partial sums of this group: plane ((group * batch + img) * nsig + s) of Py x Px
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s >= nsig) break;
      cx<float>* dst = part + (((long long)blockIdx.z * gridDim.y + img) * nsig + s) * ((long long)Py * Px);
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int e = threadIdx.x + j * nthr;
        if (e < Py * B) {
          const int u = e >> lgB, v = v0 + (e & (B - 1));
          if (v < Px) dst[(long long)u * Px + v] = Z[s][j];
        }
      }
    }
    return;
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

// The groups' partial sums added in group order, then the inverse column transform and
// the store of the ny output rows (the tail of k_conv_cols for split component loops).
template <int NB, int EPT>
__global__ void __launch_bounds__(512) k_conv_cols_sum(const cx<float>* __restrict__ part, int groups,
                                                      cx<float>* __restrict__ C, long long planeCsig,
                                                      long long planeCimg, int ldC, int ny, int Px, int nsig,
                                                      FftDesc d, const cx<float>* __restrict__ tw, int lgB) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int B = 1 << lgB, Py = d.P, nthr = blockDim.x, TF = nthr >> lgB;
  const int c = threadIdx.x & (B - 1), f = threadIdx.x >> lgB;
  const int v0 = blockIdx.x * B;
  const int img = blockIdx.y, batch = gridDim.y;
  Layout L{B, lgB, 0};
  for (int s = 0; s < nsig; ++s) {
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = threadIdx.x + j * nthr;
      if (e < Py * B) {
        const int u = e >> lgB, v = v0 + (e & (B - 1));
        cx<float> a = mk(0.f, 0.f);
        if (v < Px)
          for (int g = 0; g < groups; ++g)
            a = a + part[(((long long)g * batch + img) * nsig + s) * ((long long)Py * Px) + (long long)u * Px + v];
        buf[e] = a;
      }
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
    __syncthreads();   // buf is refilled for the next signal
  }
}

// conv_rows_inv: y = scale * Re IFFT_x(C_0), or Re IFFT_x(C_0) / Re IFFT_x(C_1).
template <int NB, int EPX>
__global__ void __launch_bounds__(512) k_conv_rows_inv(
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
// adjoint of the convolution w.r.t. the components: D_k(u, v) = sum_b Gh_b(u, v) conj(FFT_y(B_{k,b})(u, v))
// (fixed batch order, no atomics). With lacc the batch sum is kept in LDS beside the
// transform buffer (every thread owns the same elements for all b) and D is written once;
// otherwise D is read and written per image.
template <int NB>
__global__ void __launch_bounds__(512) k_grad_filter_cols(
    const cx<float>* __restrict__ Bk, long long planeBk, long long planeBimg, int ldB,
    const cx<float>* __restrict__ Gh, long long planeGimg, int ldG, cx<float>* __restrict__ D,
    long long planeDk, int ldD, int ny, int Px, int W, int batch, FftDesc d,
    const cx<float>* __restrict__ tw, int lgB, int lacc) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  cx<float>* acc = buf + ((long long)d.P << lgB);
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
        if (lacc) {
          acc[e] = b == 0 ? p : acc[e] + p;
        } else {
          cx<float>* dst = Dk + (long long)u * ldD + v;
          if (b == 0) *dst = p;
          else *dst = *dst + p;
        }
      }
    }
    __syncthreads();
  }
  if (lacc) {
    for (int e = threadIdx.x; e < Py * B; e += nthr) {
      const int u = e >> lgB, v = v0 + (e & (B - 1));
      if (v < Px) Dk[(long long)u * ldD + v] = acc[e];
    }
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
// host launchers
hipError_t launch_conv_rows_fwd(hipStream_t s, const RowCfg& c, int batch, const float* H,
                                long long planeH, int ldH, const Field& fld, int sig_norm,
                                int nsig, cx<float>* Bk, long long planeBk, long long planeBsig,
                                long long planeBimg, int ldB, int ny, int nx, int U,
                                const FftDesc& d, const cx<float>* tw) {
  if (c.B * c.TF > 512) return hipErrorInvalidValue;   // the kernel's launch bound
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
                            int nsig, const FftDesc& d, const cx<float>* tw, int groups, cx<float>* part) {
  (void)Py;
  const int B = 1 << c.lgB;
  if (groups < 1 || (groups > 1 && !part)) return hipErrorInvalidValue;
  const int per = (U + groups - 1) / groups, G = (U + per - 1) / per;
  dim3 grid((Px + B - 1) / B, batch, G), block(c.nthr);
  const size_t lds = lds_cols(c, d, sizeof(cx<float>));
  cx<float>* pp = G > 1 ? part : nullptr;
  ECC_NB_SWITCH(c.NB, ECC_EPT_SWITCH(c.EPT, hipLaunchKernelGGL((k_conv_cols<NB, EPT>), grid, block, lds, s,
                                         Bk, planeBk, planeBsig, planeBimg, ldB, Fh, planeFk, ldF,
                                         fullplane, parity, w, C, planeCsig, planeCimg, ldC, ny, Px,
                                         W, U, nsig, d, tw, c.lgB, per, pp)));
  if (G > 1) {
    hipError_t e = last();
    if (e != hipSuccess) return e;
    const dim3 g2((Px + B - 1) / B, batch);
    ECC_NB_SWITCH(c.NB, ECC_EPT_SWITCH(c.EPT, hipLaunchKernelGGL((k_conv_cols_sum<NB, EPT>), g2, block, lds, s,
                                           part, G, C, planeCsig, planeCimg, ldC, ny, Px, nsig, d, tw,
                                           c.lgB)));
  }
  return last();
}

hipError_t launch_conv_rows_inv(hipStream_t s, const RowCfg& c, int batch, const cx<float>* C,
                                long long planeCsig, long long planeCimg, int ldC, float* y,
                                long long planeY, int ldY, int ny, int nx, int nsig, float scale_,
                                const FftDesc& d, const cx<float>* tw) {
  if (c.B * c.TF > 512) return hipErrorInvalidValue;   // the kernel's launch bound
  dim3 grid((ny + c.B - 1) / c.B, batch), block(c.B * c.TF);
  const size_t lds = lds_rows(c, d, sizeof(cx<float>));
  ECC_NB_SWITCH(c.NB, ECC_EPX_SWITCH(c.EPX, hipLaunchKernelGGL((k_conv_rows_inv<NB, EPX>), grid, block, lds, s,
                                         C, planeCsig, planeCimg, ldC, y, planeY, ldY, ny, nx, nsig,
                                         scale_, d, tw, c.B, c.TF)));
  return last();
}

hipError_t launch_grad_filter_cols(hipStream_t s, const ColCfg& c, int batch,
                                   const cx<float>* Bk, long long planeBk, long long planeBimg,
                                   int ldB, const cx<float>* Gh, long long planeGimg, int ldG,
                                   cx<float>* D, long long planeDk, int ldD, int ny, int Py, int Px,
                                   int U, const FftDesc& d, const cx<float>* tw) {
  (void)Py;
  const int B = 1 << c.lgB;
  dim3 grid((Px + B - 1) / B, U), block(c.nthr);
  // the batch sum in LDS when it fits beside the transform buffer
  const size_t lds0 = lds_cols(c, d, sizeof(cx<float>));
  const size_t lds1 = lds0 + ((size_t)d.P << c.lgB) * sizeof(cx<float>);
  const int lacc = lds1 <= 160 * 1024 ? 1 : 0;
  const size_t lds = lacc ? lds1 : lds0;
  ECC_NB_SWITCH(c.NB, hipLaunchKernelGGL(k_grad_filter_cols<NB>, grid, block, lds, s, Bk, planeBk,
                                         planeBimg, ldB, Gh, planeGimg, ldG, D, planeDk, ldD, ny,
                                         Px, Px / 2 + 1, batch, d, tw, c.lgB, lacc));
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


hipError_t prepare_conv_kernels() {
  hipError_t e = hipSuccess;
#define ECC_ALLOW(...) if (e == hipSuccess) e = allow_lds(__VA_ARGS__)
#define ECC_ALLOW_NB(KN) ECC_ALLOW(KN<1>); ECC_ALLOW(KN<2>); ECC_ALLOW(KN<4>)
#define ECC_ALLOW_NB_E(KN, E) ECC_ALLOW(KN<1, E>); ECC_ALLOW(KN<2, E>); ECC_ALLOW(KN<4, E>)
#define ECC_ALLOW_EPX(KN) \
  ECC_ALLOW_NB_E(KN, 1); ECC_ALLOW_NB_E(KN, 2); ECC_ALLOW_NB_E(KN, 4); ECC_ALLOW_NB_E(KN, 8); ECC_ALLOW_NB_E(KN, 16)
  ECC_ALLOW_NB(k_grad_filter_cols);
  ECC_ALLOW_EPX(k_conv_rows_fwd);
  ECC_ALLOW_EPX(k_conv_rows_inv);
  ECC_ALLOW_NB_E(k_conv_cols, 4); ECC_ALLOW_NB_E(k_conv_cols, 8); ECC_ALLOW_NB_E(k_conv_cols, 12);
  ECC_ALLOW_NB_E(k_conv_cols, 16); ECC_ALLOW_NB_E(k_conv_cols, 24); ECC_ALLOW_NB_E(k_conv_cols, 32);
  ECC_ALLOW_NB_E(k_conv_cols_sum, 4); ECC_ALLOW_NB_E(k_conv_cols_sum, 8); ECC_ALLOW_NB_E(k_conv_cols_sum, 12);
  ECC_ALLOW_NB_E(k_conv_cols_sum, 16); ECC_ALLOW_NB_E(k_conv_cols_sum, 24); ECC_ALLOW_NB_E(k_conv_cols_sum, 32);
  return e;
}

}  // namespace ecc
