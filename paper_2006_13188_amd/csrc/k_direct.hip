// Direct (spatial) extended correlation for small filters: no transforms. For every output
// pixel p and component c,
//   G_c(p) = sum_{x in [-R, R]^2} H(p + x) conj(F_c(x))      (zero outside the image),
// combined as y(p) = scale sum_c w_c Re(e^{i (kofs + c) alpha(p)} G_c(p)): eq. Def-ECorr
// in the real-filter half form, with the standard correlations of section 4 evaluated
// as sums. It costs 2 U S^2 fused multiply-adds per pixel against a few transforms per
// component for the block path, so it pays only for the smallest filters.
//
// One workgroup of 256 threads per 16 x 64 block of outputs. The block's window of the
// signal (16 + 2R rows of 64 + 2R values, zero outside the image) sits in LDS; thread
// (r, q) owns the four pixels (y0 + r, x0 + 4q + j), j < 4, reads one window row segment of
// 4 + 2R values per filter row with 16-byte LDS reads, and accumulates its four G_c with
// two FMAs per tap. The taps are the same for the whole workgroup, so they are read through
// scalar loads (wave-uniform addresses) and enter the FMAs as scalar operands; the filter
// side is a template parameter so that every tap of a filter row has a constant offset.
#include "tile_common.hpp"

namespace ecc {

namespace {

constexpr int kDirRows = 16, kDirCols = 64, kDirThreads = 256;

template <int S>
constexpr int direct_pitch() {
  return (kDirCols + 2 * ((S - 1) / 2) + 3) & ~3;   // a multiple of 4 floats (16-byte reads)
}
template <int S>
constexpr int direct_lds_floats() {
  return (kDirRows + S - 1) * direct_pitch<S>();
}

// One block (image img, block index `tile` of a.tx x a.ty blocks of 16 x 64); a.Fs holds
// the U components as U x S x S complex64 values, F_c(x) at [c][R + x_y][R + x_x].
template <int S>
__device__ __forceinline__ void direct_block(const TileArgs& a, int img, int tile, float* win) {
  constexpr int R = (S - 1) / 2, WR = kDirRows + 2 * R, WC = kDirCols + 2 * R, WP = direct_pitch<S>();
  constexpr int NV = (4 + 2 * R + 3) / 4;   // 16-byte reads per row segment
  static_assert(4 * 15 + 4 * NV <= WP, "row segments stay inside the pitch");
  const int t = threadIdx.x, r = t / 16, q = t % 16;
  const int y0 = (tile / a.tx) * kDirRows, x0 = (tile % a.tx) * kDirCols;
  const float* Hb = a.H + (long long)img * a.planeH;

  // per-pixel phase: z = e^{i kofs alpha}, advanced by e1 = e^{i alpha} per component
  const int py = y0 + r, px = x0 + 4 * q;
  cx<float> z[4], e1[4];
  float acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    acc[j] = 0.f;
    z[j] = mk(0.f, 0.f);
    e1[j] = mk(0.f, 0.f);
    if (py < a.ny && px + j < a.nx) {
      const float fv = a.fld.ptr[(long long)img * a.fld.plane + (long long)py * a.fld.ld + px + j];
      if (a.fld.log_mode || a.kofs != 0) {
        const double al = field_angle(a.fld, fv);
        double sn, cs;
        sincos(al, &sn, &cs);
        e1[j] = mk((float)cs, (float)sn);
        sincos((double)a.kofs * al, &sn, &cs);
        z[j] = mk((float)cs, (float)sn);
      } else {
        float sn, cs;
        sincosf((float)a.fld.mul * fv + (float)a.fld.add, &sn, &cs);
        e1[j] = mk(cs, sn);
        z[j] = mk(1.f, 0.f);
      }
    }
  }
  __syncthreads();   // the window may still be in use by the previous block
  for (int e = t; e < WR * WP; e += kDirThreads) {
    const int i = e / WP, jj = e - i * WP;
    const int gy = y0 - R + i, gx = x0 - R + jj;
    win[e] = (jj < WC && gy >= 0 && gy < a.ny && gx >= 0 && gx < a.nx) ? Hb[(long long)gy * a.ldH + gx] : 0.f;
  }
  __syncthreads();

  for (int c = 0; c < a.U; ++c) {
    const cx<float>* tc = a.Fs + (long long)c * S * S;
    float gre[4] = {0.f, 0.f, 0.f, 0.f}, gim[4] = {0.f, 0.f, 0.f, 0.f};
    // (one filter row per iteration: its 2S tap values fit in scalar registers)
#pragma unroll 1
    for (int dy = 0; dy < S; ++dy) {
      float seg[4 * NV];
      const float4* src = reinterpret_cast<const float4*>(win + (r + dy) * WP + 4 * q);
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const float4 v = src[k];
        seg[4 * k] = v.x;
        seg[4 * k + 1] = v.y;
        seg[4 * k + 2] = v.z;
        seg[4 * k + 3] = v.w;
      }
      const cx<float>* trow = tc + dy * S;
#pragma unroll
      for (int dx = 0; dx < S; ++dx) {
        const cx<float> f = trow[dx];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          gre[j] = fmaf(seg[j + dx], f.re, gre[j]);
          gim[j] = fmaf(-seg[j + dx], f.im, gim[j]);   // H conj(F)
        }
      }
    }
    const float wc = a.w[c];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[j] += wc * (z[j].re * gre[j] - z[j].im * gim[j]);
      z[j] = cmul(z[j], e1[j]);
    }
  }
  float* yb = a.y + (long long)img * a.planeY;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (py < a.ny && px + j < a.nx) yb[(long long)py * a.ldY + px + j] = acc[j] * a.scale;
}

// The convolution in the same layout: y(p) = scale Re sum_c w_c sum_x M_c(p - x) F_c(x) with
// M_c(q) = H(q) e^{-i c alpha(q)} (eq. Def-EConv in the real-filter half form, the phase
// taken at the source pixel). The block's window of M_c (complex) is formed in LDS for
// every component: each thread keeps H(q) and the phase recurrence z = e^{-i c alpha(q)},
// e1 = e^{-i alpha(q)} of its share of the window pixels in registers. Output (r, 4q + j)
// with tap (dy, dx) reads M at window (r + dy, 4q + j + dx) against the flipped tap
// F_c[S - 1 - dy][S - 1 - dx] (x = (R - dy, R - dx)), Re(M F) = M.re F.re - M.im F.im.
template <int S>
constexpr int direct_cpitch() {
  return (kDirCols + S - 1 + 1) & ~1;   // complex values per window row, even (16-byte reads)
}
template <int S>
__device__ __forceinline__ void direct_conv_block(const TileArgs& a, int img, int tile, cx<float>* mw) {
  constexpr int R = (S - 1) / 2, WR = kDirRows + 2 * R, WC = kDirCols + 2 * R, WP = direct_cpitch<S>();
  constexpr int NW = (WR * WC + kDirThreads - 1) / kDirThreads;   // window pixels per thread
  constexpr int NV = (4 + 2 * R) / 2;                                 // 16-byte reads per segment
  static_assert(2 * (4 * 15 + 2 * NV) <= 2 * WP, "row segments stay inside the pitch");
  const int t = threadIdx.x, r = t / 16, q = t % 16;
  const int y0 = (tile / a.tx) * kDirRows, x0 = (tile % a.tx) * kDirCols;
  const float* Hb = a.H + (long long)img * a.planeH;
  const float* Fb = a.fld.ptr + (long long)img * a.fld.plane;
  float h[NW];
  cx<float> z[NW], e1[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int e = t + kDirThreads * k, i = e / WC, jj = e - (e / WC) * WC;
    const int gy = y0 - R + i, gx = x0 - R + jj;
    h[k] = 0.f;
    z[k] = mk(1.f, 0.f);
    e1[k] = mk(1.f, 0.f);
    if (e < WR * WC && gy >= 0 && gy < a.ny && gx >= 0 && gx < a.nx) {
      h[k] = Hb[(long long)gy * a.ldH + gx];
      const float fv = Fb[(long long)gy * a.fld.ld + gx];
      if (a.fld.log_mode) {
        double sn, cs;
        sincos(field_angle(a.fld, fv), &sn, &cs);
        e1[k] = mk((float)cs, (float)-sn);
      } else {
        float sn, cs;
        sincosf((float)a.fld.mul * fv + (float)a.fld.add, &sn, &cs);
        e1[k] = mk(cs, -sn);
      }
    }
  }
  const int py = y0 + r, px = x0 + 4 * q;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  __syncthreads();   // the window may still be in use by the previous block
  for (int c = 0; c < a.U; ++c) {
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int e = t + kDirThreads * k, i = e / WC, jj = e - (e / WC) * WC;
      if (e < WR * WC) mw[i * WP + jj] = mk(h[k] * z[k].re, h[k] * z[k].im);
      z[k] = cmul(z[k], e1[k]);
    }
    __syncthreads();
    const cx<float>* tc = a.Fs + (long long)c * S * S;
    float g[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int dy = 0; dy < S; ++dy) {
      cx<float> seg[2 * NV];
      const float4* src = reinterpret_cast<const float4*>(mw + (r + dy) * WP + 4 * q);
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const float4 v = src[k];
        seg[2 * k] = mk(v.x, v.y);
        seg[2 * k + 1] = mk(v.z, v.w);
      }
      const cx<float>* trow = tc + (S - 1 - dy) * S;
#pragma unroll
      for (int dx = 0; dx < S; ++dx) {
        const cx<float> f = trow[S - 1 - dx];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          g[j] = fmaf(seg[j + dx].re, f.re, g[j]);
          g[j] = fmaf(-seg[j + dx].im, f.im, g[j]);
        }
      }
    }
    const float wc = a.w[c];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = fmaf(wc, g[j], acc[j]);
    __syncthreads();   // the next component rewrites the window
  }
  float* yb = a.y + (long long)img * a.planeY;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (py < a.ny && px + j < a.nx) yb[(long long)py * a.ldY + px + j] = acc[j] * a.scale;
}

template <int S>
__global__ void __launch_bounds__(kDirThreads) k_direct_conv(TileArgs a) {
  __shared__ __attribute__((aligned(16))) cx<float> mw[(kDirRows + S - 1) * direct_cpitch<S>()];
  const int ntile = a.tx * a.ty;
  direct_conv_block<S>(a, blockIdx.x / ntile, blockIdx.x % ntile, mw);
}
template <int S>
__global__ void __launch_bounds__(kDirThreads) k_direct_conv_items(const TileArgs* __restrict__ descs,
                                                                  const int2* __restrict__ items) {
  __shared__ __attribute__((aligned(16))) cx<float> mw[(kDirRows + S - 1) * direct_cpitch<S>()];
  const int2 it = items[blockIdx.x];
  direct_conv_block<S>(descs[it.x], 0, it.y, mw);
}

template <int S>
__global__ void __launch_bounds__(kDirThreads) k_direct_corr(TileArgs a) {
  __shared__ __attribute__((aligned(16))) float win[direct_lds_floats<S>()];
  const int ntile = a.tx * a.ty;
  direct_block<S>(a, blockIdx.x / ntile, blockIdx.x % ntile, win);
}

// Batches: one workgroup per item (descriptor index, block index)
template <int S>
__global__ void __launch_bounds__(kDirThreads) k_direct_items(const TileArgs* __restrict__ descs,
                                                             const int2* __restrict__ items) {
  __shared__ __attribute__((aligned(16))) float win[direct_lds_floats<S>()];
  const int2 it = items[blockIdx.x];
  direct_block<S>(descs[it.x], 0, it.y, win);
}

}  // namespace

#define ECC_DIRECT_SIZES(X) X(3) X(5) X(7) X(9) X(11) X(13) X(15)

bool direct_supported(int S) {
#define ECC_DS(s_) if (S == s_) return true;
  ECC_DIRECT_SIZES(ECC_DS)
#undef ECC_DS
  return false;
}

void direct_blocks(int ny, int nx, int* tx, int* ty) {
  *tx = (nx + kDirCols - 1) / kDirCols;
  *ty = (ny + kDirRows - 1) / kDirRows;
}

hipError_t launch_direct(hipStream_t s, bool conv, int S, int batch, const TileArgs& a0) {
  TileArgs a = a0;
  direct_blocks(a.ny, a.nx, &a.tx, &a.ty);
  const long long nblk = (long long)a.tx * a.ty * batch;
  if (batch < 1 || a.U < 1 || a.R != (S - 1) / 2 || nblk > 0x7fffffffLL || (conv && a.kofs != 0))
    return hipErrorInvalidValue;
#define ECC_DL(s_)                                                                                      \
  if (S == s_) {                                                                                       \
    if (conv)                                                                                          \
      hipLaunchKernelGGL((k_direct_conv<s_>), dim3((unsigned)nblk), dim3(kDirThreads), 0, s, a);        \
    else                                                                                               \
      hipLaunchKernelGGL((k_direct_corr<s_>), dim3((unsigned)nblk), dim3(kDirThreads), 0, s, a);        \
    return last();                                                                                     \
  }
  ECC_DIRECT_SIZES(ECC_DL)
#undef ECC_DL
  return hipErrorInvalidValue;
}

hipError_t launch_direct_items(hipStream_t s, bool conv, int S, const TileArgs* descs, const int2* items,
                               int nitems) {
  if (nitems < 1) return hipErrorInvalidValue;
#define ECC_DI(s_)                                                                                      \
  if (S == s_) {                                                                                       \
    if (conv)                                                                                          \
      hipLaunchKernelGGL((k_direct_conv_items<s_>), dim3((unsigned)nitems), dim3(kDirThreads), 0, s, descs, \
                         items);                                                                       \
    else                                                                                               \
      hipLaunchKernelGGL((k_direct_items<s_>), dim3((unsigned)nitems), dim3(kDirThreads), 0, s, descs,  \
                         items);                                                                       \
    return last();                                                                                     \
  }
  ECC_DIRECT_SIZES(ECC_DI)
#undef ECC_DI
  return hipErrorInvalidValue;
}

}  // namespace ecc
