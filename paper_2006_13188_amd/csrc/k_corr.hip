// HIP kernels (gfx950) of the extended-correlation path (Sec. 4.1 of "Efficient
// Spatially Adaptive Convolution and Correlation"), for a real signal H and components
// F_k, k = 0..U-1:
//   rows_r2c   : A(i, v)   = FFT_x of H rows, half spectrum v in [0, W), W = Px/2 + 1
//   cols_fwd   : Hh(u, v)  = FFT_y of A columns (zero rows beyond ny)
//   corr_cols  : T_k(i, v) = IFFT_y(Hh conj Fh_k) cropped to i < ny, for all v in [0, Px);
//                the column Px - v comes from column v through conjugate symmetry of Hh
//   corr_rows  : y = scale * sum_k w_k Re(e^{i k alpha} IFFT_x(T_k)), cropped to nx
//   match_rows : the same row transforms, response at A equispaced angles, best angle
// All global accesses are bounds-checked against the image, spectrum and plane sizes.
#include "kcommon.hpp"

namespace ecc {

// ---------------------------------------------------------------------------------
// rows_r2c: two real rows packed as one complex transform, split after the FFT.
template <int NB>
__global__ void __launch_bounds__(512) k_rows_r2c(const float* __restrict__ H, long long planeH,
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
// A workgroup owns B adjacent columns and a chunk of components: the signal spectrum
// stays in registers for the whole chunk, and the filter spectrum of the next
// component is loaded while the current one is transformed.
template <int NB, int EPT, bool FULL>
__global__ void __launch_bounds__(1024) k_corr_cols(
    const cx<float>* __restrict__ Hh, long long planeHh, int ldHh, const cx<float>* __restrict__ Fh,
    long long planeFk, int ldF, const float* __restrict__ parity, cx<float>* __restrict__ T,
    long long planeTk, long long planeTimg, int ldT, int ny, int Px, int W, int U, int kchunk,
    int nxb, int nch, int conj_mode, FftDesc d, const cx<float>* __restrict__ tw, int lgB) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int B = 1 << lgB, Py = d.P, nthr = blockDim.x, TF = nthr >> lgB;
  const int c = threadIdx.x & (B - 1), f = threadIdx.x >> lgB;
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  const int xb = lb % nxb, rest = lb / nxb;
  const int ch = rest % nch, img = rest / nch;
  const int k0 = ch * kchunk, k1 = min(U, k0 + kchunk);
  // element j of this thread: row u = f + j*TF of column v (buf index u*B + c)
  const int v = xb * B + c;
  const bool vin = v < W;
  const int vm = (v == 0) ? 0 : Px - v;
  const cx<float>* Hb = Hh + (long long)img * planeHh;
  Layout L{B, lgB, 0};
  cx<float> h[EPT], ga[EPT], gb[FULL ? EPT : 1];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int u = f + j * TF;
    h[j] = mk(0.f, 0.f);
    ga[j] = mk(0.f, 0.f);
    if (FULL) gb[j] = mk(0.f, 0.f);
    if (u < Py && vin) {
      h[j] = Hb[u * ldHh + v];
      if (k0 < k1) {
        const cx<float>* Fk = Fh + (long long)k0 * planeFk;
        ga[j] = Fk[u * ldF + v];
        if (FULL) gb[j] = Fk[((u == 0) ? 0 : Py - u) * ldF + vm];
      }
    }
  }
  for (int k = k0; k < k1; ++k) {
    cx<float> gn[EPT], gbn[FULL ? EPT : 1];
    const bool pre = (k + 1 < k1);
    if (pre) {
      const cx<float>* Fn = Fh + (long long)(k + 1) * planeFk;
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int u = f + j * TF;
        gn[j] = mk(0.f, 0.f);
        if (FULL) gbn[j] = mk(0.f, 0.f);
        if (u < Py && vin) {
          gn[j] = Fn[u * ldF + v];
          if (FULL) gbn[j] = Fn[((u == 0) ? 0 : Py - u) * ldF + vm];
        }
      }
    }
    const float par = FULL ? 1.f : parity[k];
    cx<float>* Tk = T + (long long)img * planeTimg + (long long)k * planeTk;
    for (int half = 0; half < 2; ++half) {
      // conj_mode 0: (h conj a, h b); 1: (h a, h conj b); 2: (h b, h conj a)
      const bool use_b = (conj_mode == 2) ? (half == 0) : (half == 1);
      const bool use_conj = (conj_mode == 0) ? (half == 0) : (half == 1);
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int u = f + j * TF;
        if (u < Py) {
          cx<float> g = (FULL && use_b) ? gb[j] : ga[j];
          if (!FULL && use_b) g = scale(g, par);
          buf[(u << lgB) + c] = use_conj ? cmulc(h[j], g) : cmul(h[j], g);
        }
      }
      __syncthreads();
      run_fft<NB, +1, true, float>(buf, L, d, twl, c, f, TF, true);
      if (vin && (half == 0 || (v != 0 && 2 * v != Px))) {
        // mirror column Px - v goes to the second plane at index v
        cx<float>* dst = half == 0 ? Tk : Tk + (long long)ny * ldT;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const int i = f + j * TF;
          if (i < ny) {
            const cx<float> r = buf[(i << lgB) + c];
            dst[i * ldT + v] = half == 0 ? r : conj(r);
          }
        }
      }
      // the next product overwrites only this thread's own elements (same mapping)
    }
    if (pre) {
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        ga[j] = gn[j];
        if (FULL) gb[j] = gbn[j];
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// corr_rows: inverse row transforms of every component and the per-pixel combination
//   y = scale * sum_k w_k Re(e^{i k alpha} G_k).
// One image row per workgroup, two transforms at a time (components k = 2i and 2i+1,
// TF threads each); the rows of the next pair are loaded while the current pair is
// transformed, and the two partial sums meet in LDS at the end.
// Optional second output y2 = y2scale * mulsig * sum_k w_k k Im(e^{ik alpha} G_k) (adjoint).
template <int NB, int EPX, int EPP>
__global__ void __launch_bounds__(512) k_corr_rows(
    const cx<float>* __restrict__ T, long long planeTk, long long planeTimg, int ldT, Field fld,
    float* __restrict__ y, long long planeY, int ldY, int ny, int nx, int U,
    const float* __restrict__ w, float scl, float* __restrict__ y2,
    const float* __restrict__ mulsig, long long planeMul, int ldMul, float y2scale, int kofs,
    int accum, FftDesc d, const cx<float>* __restrict__ tw, int TF) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int Px = d.P;
  const int c = threadIdx.x / TF, f = threadIdx.x - c * TF;   // c in {0, 1}
  const int row = blockIdx.x, img = blockIdx.y;
  Layout L{2, 0, Px};
  Phase z[EPX], e2[EPX];
  float acc[EPX], acc2[EPX];
#pragma unroll
  for (int j = 0; j < EPX; ++j) {
    const int x = f + j * TF;
    z[j].re = 1.0;
    z[j].im = 0.0;
    e2[j] = z[j];
    acc[j] = 0.f;
    acc2[j] = 0.f;
    if (x < nx) {
      const double a = field_angle(fld, fld.ptr[(long long)img * fld.plane + (long long)row * fld.ld + x]);
      double sn, cs;
      sincos(a, &sn, &cs);
      Phase e1;
      e1.re = cs;
      e1.im = sn;
      e2[j] = pmul(e1, e1);
      // this transform starts at component kofs + c: e^{i (kofs + c) alpha}
      sincos((double)(kofs + c) * a, &sn, &cs);
      z[j].re = cs;
      z[j].im = sn;
    }
  }
  const cx<float>* Tb = T + (long long)img * planeTimg;
  const int W = Px / 2 + 1;
  cx<float> nxt[EPP];
#pragma unroll
  for (int j = 0; j < EPP; ++j) {
    const int pos = f + j * TF;
    nxt[j] = mk(0.f, 0.f);
    if (c < U && pos < Px) nxt[j] = stack_load(Tb + (long long)c * planeTk, row, pos, ldT, ny, W, Px);
  }
  for (int k0 = 0; k0 < U; k0 += 2) {
    const int k = k0 + c;
#pragma unroll
    for (int j = 0; j < EPP; ++j) {
      const int pos = f + j * TF;
      if (pos < Px) buf[c * Px + pos] = nxt[j];
    }
    if (k + 2 < U) {
      const cx<float>* src = Tb + (long long)(k + 2) * planeTk;
#pragma unroll
      for (int j = 0; j < EPP; ++j) {
        const int pos = f + j * TF;
        if (pos < Px) nxt[j] = stack_load(src, row, pos, ldT, ny, W, Px);
      }
    } else {
#pragma unroll
      for (int j = 0; j < EPP; ++j) nxt[j] = mk(0.f, 0.f);
    }
    __syncthreads();
    run_fft<NB, +1, false, float>(buf, L, d, twl, c, f, TF, true);
    if (k < U) {
      const float wk = w[k];
#pragma unroll
      for (int j = 0; j < EPX; ++j) {
        const int x = f + j * TF;
        if (x < nx) {
          const cx<float> g = buf[c * Px + x];
          const float zr = (float)z[j].re, zi = (float)z[j].im;
          acc[j] += wk * (zr * g.re - zi * g.im);
          if (y2) acc2[j] += wk * (float)(kofs + k) * (zr * g.im + zi * g.re);
        }
        z[j] = pmul(z[j], e2[j]);
      }
    }
  }
  __syncthreads();
  float* red = reinterpret_cast<float*>(buf);   // 4 Px floats available
  if (c == 1) {
#pragma unroll
    for (int j = 0; j < EPX; ++j) {
      const int x = f + j * TF;
      if (x < nx) {
        red[x] = acc[j];
        red[2 * Px + x] = acc2[j];
      }
    }
  }
  __syncthreads();
  if (c == 0) {
#pragma unroll
    for (int j = 0; j < EPX; ++j) {
      const int x = f + j * TF;
      if (x < nx) {
        const long long o = (long long)img * planeY + (long long)row * ldY + x;
        const float v1 = (acc[j] + red[x]) * scl;
        y[o] = accum ? y[o] + v1 : v1;
        if (y2) {
          const float v2 = (acc2[j] + red[2 * Px + x]) * scl * y2scale *
                           mulsig[(long long)img * planeMul + (long long)row * ldMul + x];
          y2[o] = accum ? y2[o] + v2 : v2;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// match_rows: response at n_angles equispaced angles, C(m) = sum_k w_k Re(e^{2 pi i k m / A} G_k),
// kept per pixel in registers; best score and the smallest maximising index. A row wider
// than the EPX TF pixels one workgroup keeps is split into segments (blockIdx.y), each
// transforming the whole row and keeping its own pixels.
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
  const int xs = blockIdx.y * EPX * TF;   // first pixel of this segment
  Layout L{B, 0, Px};
  float acc[EPX][AMAX];
#pragma unroll
  for (int j = 0; j < EPX; ++j)
#pragma unroll
    for (int m = 0; m < AMAX; ++m) acc[j][m] = 0.f;
  const int W = Px / 2 + 1;
  for (int k = 0; k < U; ++k) {
    if (active) {
      const cx<float>* src = T + (long long)k * planeTk;
      for (int pos = f; pos < Px; pos += TF) buf[c * Px + pos] = stack_load(src, row, pos, ldT, ny, W, Px);
    }
    __syncthreads();
    run_fft<NB, +1, false, float>(buf, L, d, twl, c, f, TF, active);
    const float wk = w[k];
#pragma unroll
    for (int j = 0; j < EPX; ++j) {
      const int x = xs + f + j * TF;
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
      const int x = xs + f + j * TF;
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
// host launchers
hipError_t launch_rows_r2c(hipStream_t s, const RowCfg& c, int batch, const float* H, long long planeH,
                           int ldH, cx<float>* A, long long planeA, int ldA, int ny, int nx, int W,
                           const FftDesc& d, const cx<float>* tw) {
  if (c.B * c.TF > 512) return hipErrorInvalidValue;   // the kernel's launch bound
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
  const int nxb = (W + B - 1) / B, nch = (U + kchunk - 1) / kchunk;
  dim3 grid(nxb * nch * batch), block(c.nthr);
  const size_t lds = lds_cols(c, d, sizeof(cx<float>));
  // exact elements per thread (rows f + j*TF, j < EPT)
  const int TF = c.nthr >> c.lgB;
  const int ept = (d.P + TF - 1) / TF;
  const int E = ept <= 4 ? 4 : ept <= 5 ? 5 : ept <= 6 ? 6 : ept <= 8 ? 8 : ept <= 9 ? 9 : ept <= 12 ? 12 : ept <= 16 ? 16 : -1;
  if (fullplane) {
    ECC_NB12_SWITCH(c.NB, ECC_EPC_SWITCH(E, hipLaunchKernelGGL((k_corr_cols<NB, EPT, true>), grid, block, lds, s,
                  Hh, planeHh, ldHh, Fh, planeFk, ldF, parity, T, planeTk, planeTimg, ldT, ny, Px, W, U,
                  kchunk, nxb, nch, conj_mode, d, tw, c.lgB)));
  } else {
    ECC_NB12_SWITCH(c.NB, ECC_EPC_SWITCH(E, hipLaunchKernelGGL((k_corr_cols<NB, EPT, false>), grid, block, lds, s,
                  Hh, planeHh, ldHh, Fh, planeFk, ldF, parity, T, planeTk, planeTimg, ldT, ny, Px, W, U,
                  kchunk, nxb, nch, conj_mode, d, tw, c.lgB)));
  }
  return last();
}

hipError_t launch_corr_rows(hipStream_t s, const RowCfg& c, int batch, const cx<float>* T,
                            long long planeTk, long long planeTimg, int ldT, const Field& fld,
                            float* y, long long planeY, int ldY, int ny, int nx, int U,
                            const float* w, float scale_, float* y2, const float* mulsig,
                            long long planeMul, int ldMul, float y2scale, int kofs, int accum,
                            const FftDesc& d, const cx<float>* tw) {
  // two transforms of c.TF threads per workgroup, one row each
  dim3 grid(ny, batch), block(2 * c.TF);
  const size_t lds = sizeof(cx<float>) * ((size_t)((d.twsize + 1) & ~1) + 2 * (size_t)d.P);
  const int need = (d.P + c.TF - 1) / c.TF;
  const int epp = need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : need <= 16 ? 16 : -1;
  ECC_NB_SWITCH(c.NB, ECC_EPX_SWITCH(c.EPX, ECC_EPP_SWITCH(epp, hipLaunchKernelGGL((k_corr_rows<NB, EPX, EPP>), grid, block, lds, s,
                                         T, planeTk, planeTimg, ldT, fld, y, planeY, ldY, ny, nx, U,
                                         w, scale_, y2, mulsig, planeMul, ldMul, y2scale, kofs,
                                         accum, d, tw, c.TF))));
  return last();
}

hipError_t launch_match_rows(hipStream_t s, const RowCfg& c, const cx<float>* T, long long planeTk,
                             int ldT, float* score, int* index, int ldOut, int ny, int nx, int U,
                             const float* w, float scale_, int n_angles, const float* angle_tab,
                             const FftDesc& d, const cx<float>* tw) {
  if (c.EPX < 1 || c.TF < 1) return hipErrorInvalidValue;
  const int nseg = (nx + c.EPX * c.TF - 1) / (c.EPX * c.TF);   // row segments (wide images)
  if (nseg > 65535) return hipErrorInvalidValue;
  dim3 grid((ny + c.B - 1) / c.B, nseg), block(c.B * c.TF);
  const size_t lds = lds_rows(c, d, sizeof(cx<float>)) + 64 * sizeof(cx<float>);
  ECC_NB_SWITCH(c.NB, ECC_EPX_SWITCH(c.EPX, hipLaunchKernelGGL((k_match_rows<NB, EPX>), grid, block, lds, s,
                                         T, planeTk, ldT, score, index, ldOut, ny, nx, U, w, scale_,
                                         n_angles, angle_tab, d, tw, c.B, c.TF)));
  return last();
}


hipError_t prepare_corr_kernels() {
  hipError_t e = hipSuccess;
#define ECC_ALLOW(...) if (e == hipSuccess) e = allow_lds(__VA_ARGS__)
#define ECC_ALLOW_NB(KN) ECC_ALLOW(KN<1>); ECC_ALLOW(KN<2>); ECC_ALLOW(KN<4>)
#define ECC_ALLOW_NB_E(KN, E) ECC_ALLOW(KN<1, E>); ECC_ALLOW(KN<2, E>); ECC_ALLOW(KN<4, E>)
#define ECC_ALLOW_EPX(KN) \
  ECC_ALLOW_NB_E(KN, 1); ECC_ALLOW_NB_E(KN, 2); ECC_ALLOW_NB_E(KN, 4); ECC_ALLOW_NB_E(KN, 8); ECC_ALLOW_NB_E(KN, 16)
  ECC_ALLOW_NB(k_rows_r2c);
  ECC_ALLOW_NB(k_cols_fwd);
#define ECC_ALLOW_CC(E) ECC_ALLOW(k_corr_cols<1, E, false>); ECC_ALLOW(k_corr_cols<2, E, false>); \
  ECC_ALLOW(k_corr_cols<1, E, true>); ECC_ALLOW(k_corr_cols<2, E, true>)
  ECC_ALLOW_CC(4); ECC_ALLOW_CC(5); ECC_ALLOW_CC(6); ECC_ALLOW_CC(8); ECC_ALLOW_CC(9); ECC_ALLOW_CC(12); ECC_ALLOW_CC(16);
#define ECC_ALLOW_CR(E, P) ECC_ALLOW(k_corr_rows<1, E, P>); ECC_ALLOW(k_corr_rows<2, E, P>); ECC_ALLOW(k_corr_rows<4, E, P>)
#define ECC_ALLOW_CRP(E) ECC_ALLOW_CR(E, 1); ECC_ALLOW_CR(E, 2); ECC_ALLOW_CR(E, 4); ECC_ALLOW_CR(E, 8); ECC_ALLOW_CR(E, 16)
  ECC_ALLOW_CRP(1); ECC_ALLOW_CRP(2); ECC_ALLOW_CRP(4); ECC_ALLOW_CRP(8); ECC_ALLOW_CRP(16);
  ECC_ALLOW_EPX(k_match_rows);
  return e;
}

}  // namespace ecc
