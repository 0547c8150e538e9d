// Tiled (overlap-save) extended convolution: every workgroup owns one T x T block of
// output pixels and computes it on chip.
//
// For component c the block's N x N window of the modulated signal
// m_c(q) = s(q) e^{-i c alpha(q)} (q = (y0 - R + i, x0 - R + j), zero outside the image) is
// transformed, multiplied by the block spectrum of F_c and accumulated over components
// with the weights w_c in the frequency domain (one register accumulator per frequency
// bin, owned by the same thread for all components); one inverse transform at the end
// gives y = Re sum_c w_c (m_c * F_c) (section 4, extended convolution by Fourier-domain
// products). F_c is placed at circular index (x - R) mod N for its offsets x in [-R, R],
// so circular output index u < N - 2R is the linear convolution at y0 + u.
//
// With two signals (scale group, ratio form of eq. normalization) the kernel runs twice:
// first for the numerator signal H / f^2 (raw real parts written), then for the
// denominator signal 1 / f^2, dividing the stored numerator by its own result. (Two
// launches rather than one block doing both: the per-thread state of one signal already
// fills the register file at N = 128.)
#include <type_traits>

#include "tile_common.hpp"

namespace ecc {

namespace {

// LDS copy of the block spectrum of one component: for N <= 96 it fits beside the
// transform image (2 x 75 KB for N = 96), and the plane is brought in by direct
// memory-to-LDS loads (1 KB per wave instruction) issued at the start of the component's
// forward transform, so that its latency is hidden behind three transform passes. A
// separate LDS object, so that the compiler can tell its loads from the image's.
constexpr bool tconv_dma(int N) { return N <= 96; }
template <int N>
__shared__ cx<float> conv_spec_lds[tconv_plane(N)];

template <int N, int NT>
__device__ __forceinline__ void stream_spectrum(const cx<float>* src) {
  constexpr int NCH = tconv_plane(N) / 128;   // 1 KB pieces: 64 lanes x 16 bytes
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int ch = w; ch < NCH; ch += NT / 64)
    __builtin_amdgcn_global_load_lds(static_cast<const void*>(src + ch * 128 + 2 * lane),
                                     (__attribute__((address_space(3))) void*)(conv_spec_lds<N> + ch * 128),
                                     16, 0, 0);
}

// Seed of scale mode l (joint plans): z = sig(q) e^{-i (k0 alpha(q) + omega_l ln s(q))} for
// this thread's window pixels, k0 = 1 for l < 0 (the half set has no (0, l < 0)), else 0;
// e1 = e^{-i alpha} is already in registers. The thread index comes in through an empty asm
// so that the addresses are formed here rather than kept live across the component loop.
template <int N, int NT, int NQ0>
__device__ __forceinline__ void joint_seed(const TileConvArgs& a, int img, int y0, int x0, int l,
                                           const cx<float> (&e1)[NQ0][8], cx<float> (&z)[NQ0][8]) {
  constexpr int M = N / 8;
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  const float* Hb = a.H + (long long)img * a.planeH;
  const float* Sb = a.jscale + (long long)img * a.plane_s;
  const float om = a.joint_om1 * (float)l;
  const bool den = a.step == 2;
#pragma unroll
  for (int s = 0; s < NQ0; ++s) {
    const int q = t + s * NT;
    const int v = q % N, b = q / N;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int gy = y0 - a.R + b + M * r, gx = x0 - a.R + v;
      z[s][r] = mk(0.f, 0.f);
      if (b < M && gy >= 0 && gy < a.ny && gx >= 0 && gx < a.nx) {
        const float sv = Sb[(long long)gy * a.ld_s + gx];
        float sn, cs;
        sincosf(om * logf(sv), &sn, &cs);
        cx<float> p = mk(cs, -sn);
        if (l < 0) p = cmul(p, e1[s][r]);
        const float wn = a.sig_norm ? 1.f / (sv * sv) : 1.f;
        const float sig = den ? wn : Hb[(long long)gy * a.ldH + gx] * wn;
        z[s][r] = mk(sig * p.re, sig * p.im);
      }
    }
  }
}

// NT threads (512 or 768); LS = NT / 8 threads share each pass-1 butterfly index.
// JOINT: the components of a joint rotation and scale plan, taken by scale mode l
// (l = -h .. h, then k = k0 .. K within a mode, so that the phase of one mode advances by
// e^{-i alpha} as for a rotation plan); component (k, l) is entry k = 0 ? l :
// h + 1 + (k - 1) n + (l + h) of the plan's half set.
template <int N, int TV, int NT, bool JOINT = false>
__device__ __forceinline__ void conv_block_one(const TileConvArgs& a, int img, int tile, cx<float>* A) {
  constexpr int M = N / 8, P = N + 1, LS = NT / 8;
  constexpr bool DMA = tconv_dma(N);
  constexpr int FP = tconv_pitch(N), FPL = tconv_plane(N);
  constexpr int NQ0 = (N * M + NT - 1) / NT;   // column pass-0 items
  constexpr int NI = (N + LS - 1) / LS;        // pass-1 lines per thread (line < N checked)
  constexpr int TR = (TV + LS - 1) / LS, RV = TV / 8;
  const int t = threadIdx.x, l = t % LS;
  // with 512 threads the butterfly index is the wave index: uniform, so its twiddles sit
  // in scalar registers (with 768 a wave straddles two indices)
  const int bq = NT == 512 ? __builtin_amdgcn_readfirstlane(t / LS) : t / LS;
  const int y0 = (tile / a.tx) * a.T, x0 = (tile % a.tx) * a.T;
  const int T = a.T;
  const TileTwiddles<N>& tt = tile_twiddles<N>();
  cx<float> tw[M];
#pragma unroll
  for (int r = 0; r < M; ++r) tw[r] = mk(tt.re[bq][r], tt.im[bq][r]);

  float out0[TR][RV];
  const float* Hb = a.H + (long long)img * a.planeH;
  const bool den = a.step == 2;   // the denominator signal 1 / f^2 (no image)
  __syncthreads();   // the LDS image may still be in use by the previous block
  {
    // ---- window pixels of this thread's column pass-0 items: z = s(q) e^{-i c alpha(q)}
    // for the current component c (starting at c = 0), advanced by e1 = e^{-i alpha}
    cx<float> z[NQ0][8], e1[NQ0][8];
#pragma unroll
    for (int s = 0; s < NQ0; ++s) {
      const int q = t + s * NT;
      const int v = q % N, b = q / N;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int gy = y0 - a.R + b + M * r, gx = x0 - a.R + v;
        z[s][r] = mk(0.f, 0.f);
        e1[s][r] = mk(0.f, 0.f);
        if (b < M && gy >= 0 && gy < a.ny && gx >= 0 && gx < a.nx) {
          const float fv = a.fld.ptr[(long long)img * a.fld.plane + (long long)gy * a.fld.ld + gx];
          float sn, cs;
          if (a.fld.log_mode) {
            double dsn, dcs;
            sincos(field_angle(a.fld, fv), &dsn, &dcs);
            sn = (float)dsn;
            cs = (float)dcs;
          } else {
            sincosf((float)a.fld.mul * fv + (float)a.fld.add, &sn, &cs);
          }
          e1[s][r] = mk(cs, -sn);
          if constexpr (!JOINT) {
            const float wn = a.sig_norm ? 1.f / (fv * fv) : 1.f;
            z[s][r] = mk(den ? wn : Hb[(long long)gy * a.ldH + gx] * wn, 0.f);
          }
        }
      }
    }
    cx<float> Z[NI][M];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int r = 0; r < M; ++r) Z[i][r] = mk(0.f, 0.f);

    // joint plans: scale mode index li = l + h and angular frequency kk of the next component
    // (with K = 0 the modes l < 0 have no components: the walk starts at l = 0)
    const int jh = JOINT ? (a.joint_n - 1) / 2 : 0;
    int li = (JOINT && a.joint_K == 0) ? jh : 0, kk = li < jh ? 1 : 0;
    for (int c = 0; c < a.U; ++c) {
      int ci = c;
      if constexpr (JOINT) {
        const int l = li - jh;
        if (kk == (l < 0 ? 1 : 0)) joint_seed<N, NT, NQ0>(a, img, y0, x0, l, e1, z);
        ci = kk == 0 ? l : jh + 1 + (kk - 1) * a.joint_n + li;
        if (++kk > a.joint_K) {
          ++li;
          kk = li - jh < 0 ? 1 : 0;
        }
      }
      const cx<float>* Fc = a.Fs + (long long)ci * FPL;
      if constexpr (DMA) stream_spectrum<N, NT>(Fc);
      const float wc = a.w[ci];
      // ---- forward transform of m_c: column pass 0 from registers
#pragma unroll
      for (int s = 0; s < NQ0; ++s) {
        const int q = t + s * NT;
        const int v = q % N, b = q / N;
        if (b < M) {
          cx<float> x[8];
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            x[r] = z[s][r];
            z[s][r] = cmul(z[s][r], e1[s][r]);
          }
          dft<8, -1, float>(x);
#pragma unroll
          for (int r = 0; r < 8; ++r) A[(8 * b + r) * P + v] = x[r];
        }
      }
      // (barriers for LDS data only: the spectrum copy stays in flight across them)
      lds_barrier();
      pass1_inplace<N, -1, false, NI, NT>(A, tw, bq, l, N, N);
      lds_barrier();
      pass0_inplace<N, -1, true, N, NT, true>(A, t, N, true);
      if constexpr (DMA) __builtin_amdgcn_s_waitcnt(0);   // this wave's spectrum pieces are in LDS
      __syncthreads();
      // ---- row pass 1 and the weighted product with the filter spectrum
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int u = l + LS * i;
        if (N % LS == 0 || u < N) {
          cx<float> x[M];
#pragma unroll
          for (int r = 0; r < M; ++r) x[r] = A[u * P + bq + 8 * r];
#pragma unroll
          for (int r = 1; r < M; ++r) x[r] = cmulc(x[r], tw[r]);
          dft<M, -1, float>(x);
#pragma unroll
          for (int r = 0; r < M; ++r) {
            const cx<float> pr = cmul(x[r], DMA ? conv_spec_lds<N>[u * FP + bq + 8 * r] : Fc[u * FP + bq + 8 * r]);
            Z[i][r].re += wc * pr.re;
            Z[i][r].im += wc * pr.im;
          }
        }
      }
      __syncthreads();   // the image is rewritten next
    }

    // ---- inverse transform; real parts of the T x T block
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int r = 0; r < M; ++r)
        if (N % LS == 0 || l + LS * i < N) A[(l + LS * i) * P + bq + 8 * r] = Z[i][r];
    __syncthreads();
    pass0_inplace<N, +1, false, N, NT>(A, t, N, true);
    __syncthreads();
    pass1_inplace<N, +1, false, NI, NT, TV / 8>(A, tw, bq, l, N, T);
    __syncthreads();
    pass0_inplace<N, +1, true, TV, NT>(A, t, T, true);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const int u = l + LS * i;
      cx<float> x[M];
#pragma unroll
      for (int r = 0; r < M; ++r) x[r] = (u < T) ? A[u * P + bq + 8 * r] : mk(0.f, 0.f);
#pragma unroll
      for (int r = 1; r < M; ++r) x[r] = cmul(x[r], tw[r]);
      dft<M, +1, float>(x);
#pragma unroll
      for (int r = 0; r < RV; ++r) out0[i][r] = x[r].re;
    }
    __syncthreads();
  }
  // outputs through LDS (the image is free after the last barrier), then stored with
  // consecutive lanes along rows (a wave's lanes above are rows of one column)
  constexpr int FL = TV + 1, FPT = (TV * TV + NT - 1) / NT;
  float* ob = reinterpret_cast<float*>(A);
#pragma unroll
  for (int i = 0; i < TR; ++i) {
#pragma unroll
    for (int r = 0; r < RV; ++r) {
      const int u = l + LS * i;
      if (u < TV) ob[u * FL + bq + 8 * r] = a.step == 0 ? out0[i][r] * a.scale : out0[i][r];
    }
  }
  __syncthreads();
  float* yb = a.y + (long long)img * a.planeY;
#pragma unroll
  for (int k = 0; k < FPT; ++k) {
    const int e = t + NT * k, row = e / TV, col = e % TV;
    const int gy = y0 + row, gx = x0 + col;
    if (e < TV * TV && row < T && col < T && gy < a.ny && gx < a.nx) {
      float* yp = yb + (long long)gy * a.ldY + gx;
      *yp = den ? *yp / ob[row * FL + col] : ob[row * FL + col];   // numerator / denominator
    }
  }
}

// Filter part of the adjoint, one block: the block's gradient g (window rows/columns
// [R, R + T), zero elsewhere) is transformed once and kept in registers as
// G'(w) = G(w) e^{-2 pi i (w_y + w_x) R / N} (the phase shifts the lags by R, so that the
// lags [-R, R] become the first S = 2R + 1 circular indices); per component the modulated
// window m_k = H e^{-ik alpha} is transformed forward as in the convolution, the product
// G' conj(M_k) is transformed back with only the first S rows and columns formed, and the
// S x S lags are written to the block's partial sums.
template <int N, int TV, int NT>
__device__ __forceinline__ void gradf_block(const TileGradFArgs& a, int img, int tile, int blk, cx<float>* A) {
  constexpr int M = N / 8, P = N + 1, LS = NT / 8;
  constexpr int NQ0 = (N * M + NT - 1) / NT;
  constexpr int NI = (N + LS - 1) / LS;
  const int t = threadIdx.x, l = t % LS;
  const int bq = NT == 512 ? __builtin_amdgcn_readfirstlane(t / LS) : t / LS;
  const int y0 = (tile / a.tx) * a.T, x0 = (tile % a.tx) * a.T;
  const int S = 2 * a.R + 1;
  const TileTwiddles<N>& tt = tile_twiddles<N>();
  cx<float> tw[M];
#pragma unroll
  for (int r = 0; r < M; ++r) tw[r] = mk(tt.re[bq][r], tt.im[bq][r]);

  __syncthreads();   // the LDS image may still be in use by the previous block
  // ---- spectrum of the block's gradient (window rows y0 - R + i; only the block is nonzero)
  forward_window<N, NT>(A, a.G + (long long)img * a.planeG, a.ldG, min(a.ny, y0 + a.T), min(a.nx, x0 + a.T),
                        y0, x0, a.R, t, y0, x0);
  const TilePhases<N>& ph = tile_phases<N>();
  cx<float> gs[NI][M];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int r = 0; r < M; ++r) {
      const int u = l + LS * i, v = bq + 8 * r;
      gs[i][r] = mk(0.f, 0.f);
      if (N % LS == 0 || u < N) {
        const int m = ((u + v) * a.R) % N;
        gs[i][r] = cmulc(window_spectrum<N>(A, u, v), mk(ph.re[m], ph.im[m]));
      }
    }
  // ---- window pixels of this thread's column pass-0 items: z = H(q) e^{-i c alpha(q)}
  const float* Hb = a.H + (long long)img * a.planeH;
  cx<float> z[NQ0][8], e1[NQ0][8];
#pragma unroll
  for (int s = 0; s < NQ0; ++s) {
    const int q = t + s * NT;
    const int v = q % N, b = q / N;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int gy = y0 - a.R + b + M * r, gx = x0 - a.R + v;
      z[s][r] = mk(0.f, 0.f);
      e1[s][r] = mk(0.f, 0.f);
      if (b < M && gy >= 0 && gy < a.ny && gx >= 0 && gx < a.nx) {
        const float fv = a.fld.ptr[(long long)img * a.fld.plane + (long long)gy * a.fld.ld + gx];
        float sn, cs;
        if (a.fld.log_mode) {
          double dsn, dcs;
          sincos(field_angle(a.fld, fv), &dsn, &dcs);
          sn = (float)dsn;
          cs = (float)dcs;
        } else {
          sincosf((float)a.fld.mul * fv + (float)a.fld.add, &sn, &cs);
        }
        e1[s][r] = mk(cs, -sn);
        z[s][r] = mk(Hb[(long long)gy * a.ldH + gx], 0.f);
      }
    }
  }
  __syncthreads();   // A is rewritten below

  cx<float>* out = a.part + (long long)blk * a.U * S * S;
  for (int c = 0; c < a.U; ++c) {
    // ---- forward transform of m_c (column pass 0 from registers)
#pragma unroll
    for (int s = 0; s < NQ0; ++s) {
      const int q = t + s * NT;
      const int v = q % N, b = q / N;
      if (b < M) {
        cx<float> x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          x[r] = z[s][r];
          z[s][r] = cmul(z[s][r], e1[s][r]);
        }
        dft<8, -1, float>(x);
#pragma unroll
        for (int r = 0; r < 8; ++r) A[(8 * b + r) * P + v] = x[r];
      }
    }
    __syncthreads();
    pass1_inplace<N, -1, false, NI, NT>(A, tw, bq, l, N, N);
    __syncthreads();
    pass0_inplace<N, -1, true, N, NT>(A, t, N, true);
    __syncthreads();
    // ---- row pass 1, then the product G' conj(M_c) in place
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int u = l + LS * i;
      if (N % LS == 0 || u < N) {
        cx<float> x[M];
#pragma unroll
        for (int r = 0; r < M; ++r) x[r] = A[u * P + bq + 8 * r];
#pragma unroll
        for (int r = 1; r < M; ++r) x[r] = cmulc(x[r], tw[r]);
        dft<M, -1, float>(x);
#pragma unroll
        for (int r = 0; r < M; ++r) A[u * P + bq + 8 * r] = cmulc(gs[i][r], x[r]);
      }
    }
    __syncthreads();
    // ---- inverse transform, first S rows and columns only
    pass0_inplace<N, +1, false, N, NT>(A, t, N, true);
    __syncthreads();
    pass1_inplace<N, +1, false, NI, NT>(A, tw, bq, l, N, S);
    __syncthreads();
    pass0_inplace<N, +1, true, N, NT>(A, t, S, true);
    __syncthreads();
    cx<float>* oc = out + (long long)c * S * S;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int u = l + LS * i;
      if (u < S) {
        cx<float> x[M];
#pragma unroll
        for (int r = 0; r < M; ++r) x[r] = A[u * P + bq + 8 * r];
#pragma unroll
        for (int r = 1; r < M; ++r) x[r] = cmul(x[r], tw[r]);
        dft<M, +1, float>(x);
#pragma unroll
        for (int r = 0; r < M; ++r)
          if (bq + 8 * r < S) oc[u * S + bq + 8 * r] = x[r];
      }
    }
    __syncthreads();   // the image is rewritten by the next component
  }
}

// threads per workgroup of the convolution: 768 for N = 96 (three waves per SIMD; the 96
// rows x 8 butterflies of the pass-1 phases are exactly one item per thread), else 512
template <int N>
constexpr int tconv_threads() {
  return N == 96 ? 768 : 512;
}
// the filter-gradient kernel keeps 512 (two waves per SIMD)
constexpr int tgradf_threads() { return 512; }

// the transform image: a static LDS object of its own (with the spectrum copy beside it
// for N <= 96), so that the compiler orders the spectrum's memory-to-LDS loads only
// against the spectrum's reads
template <int N>
__shared__ cx<float> conv_img_lds[N * (N + 1)];

template <int N, int TV>
__global__ void __launch_bounds__(tgradf_threads()) k_tile_gradf(TileGradFArgs a) {
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  const int ntile = a.tx * a.ty;
  gradf_block<N, TV, tgradf_threads()>(a, lb / ntile, lb % ntile, lb, conv_img_lds<N>);
}

// Sum of the block partials in a fixed order, in two stages: stage 1, thread (value, chunk)
// adds the blocks of its chunk in block order (float64); stage 2 adds the chunks in order.
constexpr int kGradfChunks = 64;
__global__ void k_gradf_partial(const cx<float>* __restrict__ part, int nblk, int n, cx<double>* __restrict__ tmp) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x, ch = blockIdx.y;
  if (idx >= n) return;
  const int b0 = (int)((long long)nblk * ch / kGradfChunks), b1 = (int)((long long)nblk * (ch + 1) / kGradfChunks);
  double re = 0.0, im = 0.0;
#pragma unroll 4
  for (int b = b0; b < b1; ++b) {
    const cx<float> v = part[(long long)b * n + idx];
    re += v.re;
    im += v.im;
  }
  tmp[(long long)ch * n + idx] = mk(re, im);
}
__global__ void k_gradf_final(const cx<double>* __restrict__ tmp, int n, int S, const float* __restrict__ w,
                              float scale, cx<float>* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  double re = 0.0, im = 0.0;
  for (int ch = 0; ch < kGradfChunks; ++ch) {
    const cx<double> v = tmp[(long long)ch * n + idx];
    re += v.re;
    im += v.im;
  }
  const double f = (double)w[idx / (S * S)] * scale;
  out[idx] = mk((float)(re * f), (float)(im * f));
}

template <int N, int TV, bool JOINT = false>
__global__ void __launch_bounds__(tconv_threads<N>()) k_tile_conv(TileConvArgs a) {
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  const int ntile = a.tx * a.ty;
  conv_block_one<N, TV, tconv_threads<N>(), JOINT>(a, lb / ntile, lb % ntile, conv_img_lds<N>);
}


// Batches: one workgroup per item (descriptor, block) of a list ordered by decreasing
// cost (the dispatcher starts workgroups in order, so the longest go first).
template <int N, int TV>
__global__ void __launch_bounds__(tconv_threads<N>()) k_tile_conv_items(const TileConvArgs* __restrict__ descs,
                                                                      const int2* __restrict__ items) {
  const int2 it = items[blockIdx.x];
  conv_block_one<N, TV, tconv_threads<N>()>(descs[it.x], 0, it.y, conv_img_lds<N>);
}

}  // namespace

#define ECC_TCONV_CONFIGS(X) X(64, 64) X(96, 64) X(128, 64) X(128, 96)

bool tconv_supported(int N, int TV) {
#define ECC_CS(n, tv) if (N == n && TV == tv) return true;
  ECC_TCONV_CONFIGS(ECC_CS)
#undef ECC_CS
  return false;
}

hipError_t launch_tile_conv(hipStream_t s, int N, int TV, int batch, const TileConvArgs& a0) {
  TileConvArgs a = a0;
  if (a.T < 1 || a.T > TV || a.T > N - 2 * a.R || (a.nsig != 1 && a.nsig != 2)) return hipErrorInvalidValue;
  a.tx = (a.nx + a.T - 1) / a.T;
  a.ty = (a.ny + a.T - 1) / a.T;
  const long long nblk = (long long)a.tx * a.ty * batch;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool joint = a.joint_n > 0;
  if (joint && (a.joint_n % 2 == 0 || a.joint_K < 0 || !a.jscale ||
                a.U != (a.joint_K + 1) * a.joint_n - (a.joint_n - 1) / 2))
    return hipErrorInvalidValue;
  // nsig = 2: the numerator pass, then the denominator pass dividing into it
#define ECC_CL(n, tv)                                                                              \
  if (N == n && TV == tv) {                                                                       \
    for (int step = (a.nsig == 1 ? 0 : 1); step <= (a.nsig == 1 ? 0 : 2); ++step) {              \
      a.step = step;                                                                              \
      if (joint)                                                                                  \
        hipLaunchKernelGGL((k_tile_conv<n, tv, true>), dim3((unsigned)nblk),                      \
                           dim3(tconv_threads<n>()), 0, s, a);                                    \
      else                                                                                        \
        hipLaunchKernelGGL((k_tile_conv<n, tv>), dim3((unsigned)nblk), dim3(tconv_threads<n>()),  \
                           0, s, a);                                                              \
      const hipError_t e = last();                                                                \
      if (e != hipSuccess) return e;                                                              \
    }                                                                                             \
    return hipSuccess;                                                                            \
  }
  ECC_TCONV_CONFIGS(ECC_CL)
#undef ECC_CL
  return hipErrorInvalidValue;
}

hipError_t launch_tile_conv_items(hipStream_t s, int N, int TV, const TileConvArgs* descs, const int2* items,
                                  int nitems) {
  if (nitems < 1) return hipErrorInvalidValue;
#define ECC_CI(n, tv)                                                                                 \
  if (N == n && TV == tv) {                                                                          \
    hipLaunchKernelGGL((k_tile_conv_items<n, tv>), dim3((unsigned)nitems), dim3(tconv_threads<n>()), 0, s, \
                       descs, items);                                                                \
    return last();                                                                                   \
  }
  ECC_TCONV_CONFIGS(ECC_CI)
#undef ECC_CI
  return hipErrorInvalidValue;
}

bool tgradf_supported(int N, int TV) { return tconv_supported(N, TV); }

hipError_t launch_tile_gradf(hipStream_t s, int N, int TV, int batch, const TileGradFArgs& a0) {
  TileGradFArgs a = a0;
  if (a.T < 1 || a.T > TV || a.T > N - 2 * a.R || a.R < 0) return hipErrorInvalidValue;
  a.tx = (a.nx + a.T - 1) / a.T;
  a.ty = (a.ny + a.T - 1) / a.T;
  const long long nblk = (long long)a.tx * a.ty * batch;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
#define ECC_GL(n, tv)                                                                                     \
  if (N == n && TV == tv) {                                                                              \
    hipLaunchKernelGGL((k_tile_gradf<n, tv>), dim3((unsigned)nblk), dim3(tgradf_threads()), 0, s, a);    \
    return last();                                                                                       \
  }
  ECC_TCONV_CONFIGS(ECC_GL)
#undef ECC_GL
  return hipErrorInvalidValue;
}

size_t gradf_reduce_scratch(int U, int S) { return (size_t)kGradfChunks * U * S * S * sizeof(cx<double>); }

hipError_t launch_gradf_reduce(hipStream_t s, const cx<float>* part, int nblk, int U, int S, const float* w,
                               float scale, cx<float>* out, void* scratch) {
  const int n = U * S * S;
  cx<double>* tmp = static_cast<cx<double>*>(scratch);
  hipLaunchKernelGGL(k_gradf_partial, dim3((unsigned)((n + 255) / 256), kGradfChunks), dim3(256), 0, s, part,
                     nblk, n, tmp);
  hipError_t e = last();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gradf_final, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tmp, n, S, w, scale, out);
  return last();
}

// LDS per workgroup (all static: the transform image, and the spectrum copy for N <= 96)
size_t tconv_lds_bytes(int N) {
  return (size_t)N * (N + 1) * sizeof(cx<float>) +
         (tconv_dma(N) ? (size_t)tconv_plane(N) * sizeof(cx<float>) : 0);
}

// the kernels use static LDS only: nothing to set up
hipError_t prepare_tconv_kernels() { return hipSuccess; }

}  // namespace ecc
