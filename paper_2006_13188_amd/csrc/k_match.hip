// Angle search of rotation-invariant matching over a component stack (section 5 in the
// band-limited form): for every pixel p and angle m < A,
//   C(p, m) = sum_c Re(e^{2 pi i c m / A} w_c G_c(p))
//           = sum_k D[m][k] g_k(p),  g = (Re G_0, Im G_0, Re G_1, ...),
//   D[m][2c] = w_c cos(2 pi c m / A),  D[m][2c+1] = -w_c sin(2 pi c m / A),
// a dense [A x 2U] by [2U x pixels] product, then the maximum over m and the first m
// attaining it. Three forms:
//   * float32, one thread per pixel: for A = 64 (the usual angle count) as the real-output
//     length-64 transform of the U nonzero inputs w_c G_c (one 32-point DFT, below), else
//     as fused multiply-adds with the table;
//   * matrix cores (16x16x16 MFMA) with float16 operands split into hi + lo parts:
//     D g = D_hi g_hi + D_hi g_lo + D_lo g_hi (the lo*lo term, ~2^-22 relative, dropped),
//     accumulated in float32; g is scaled per group of 16 pixels by a power of two so
//     that its largest magnitude lies in [2^10, 2^11) (lo parts stay normal numbers);
//   * the same with bfloat16 hi + lo parts (about 2^-16 relative per product).
#include "kcommon.hpp"
#include "mfma_split.hpp"

namespace ecc {

namespace {

// The stack holds U planes of npix complex values (component-major), `pitch` apart.
// UMAX >= U (the components beyond U are zero and their products are not formed past
// UMAX); the table rows of the A angles are staged in LDS (read as broadcasts).
template <int UMAX>
__global__ void __launch_bounds__(256) k_match_angles_f32(const float2* __restrict__ stack, int U,
                                                          long long npix, long long pitch, int A,
                                                          const float* __restrict__ dtab,
                                                          float* __restrict__ score, int* __restrict__ index,
                                                          int ldOut, int nx) {
  constexpr int K2 = 2 * UMAX;
  __shared__ float dl[64 * K2];
  for (int i = threadIdx.x; i < A * K2; i += 256) dl[i] = dtab[(i / K2) * 64 + i % K2];
  __syncthreads();
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  if (p >= npix) return;
  float g[K2];
#pragma unroll
  for (int c = 0; c < UMAX; ++c) {
    const float2 v = (c < U) ? stack[c * pitch + p] : make_float2(0.f, 0.f);
    g[2 * c] = v.x;
    g[2 * c + 1] = v.y;
  }
  float best = -INFINITY;
  int bi = 0;
#pragma unroll 2
  for (int m = 0; m < A; ++m) {
    const float* d = dl + m * K2;
    float c = 0.f;
#pragma unroll
    for (int k = 0; k < K2; ++k) c = fmaf(g[k], d[k], c);
    if (c > best) {
      best = c;
      bi = m;
    }
  }
  const long long y = p / nx, x = p - y * nx;
  score[y * ldOut + x] = best;
  index[y * ldOut + x] = bi;
}

// A = 64, U <= UMAX <= 32: C(m) = Re sum_c X_c e^{2 pi i c m / 64}, X_c = w_c G_c (the
// weights w_c are row m = 0 of the table). C is the length-64 transform of the Hermitian
// sequence H_0 = Re X_0, H_c = X_c / 2 and H_{64-c} = conj(X_c) / 2 (0 < c < U), whose
// output is real; as for any real-output transform, its even and odd samples are the real
// and imaginary parts of one 32-point transform:
//   C(2n) + i C(2n+1) = sum_{k<32} Z_k e^{2 pi i k n / 32},  Z_k = E_k + i O_k,
//   E_k = H_k + conj(H_{32-k}),  O_k = (H_k - conj(H_{32-k})) e^{2 pi i k / 64}  (H_32 = 0),
// about half the arithmetic of transforming the complex inputs at all 64 angles.
template <int UMAX>
__global__ void __launch_bounds__(256) k_match_angles_f32_dft64(const float2* __restrict__ stack, int U,
                                                                long long npix, long long pitch,
                                                                const float* __restrict__ dtab,
                                                                float* __restrict__ score, int* __restrict__ index,
                                                                int ldOut, int nx) {
  static_assert(UMAX <= 32, "inputs below the 32nd frequency");
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  if (p >= npix) return;
  cx<float> H[UMAX];
#pragma unroll
  for (int c = 0; c < UMAX; ++c) {
    const float2 v = (c < U) ? stack[c * pitch + p] : make_float2(0.f, 0.f);
    const float w = (c < U) ? dtab[2 * c] : 0.f;
    H[c] = c == 0 ? mk(w * v.x, 0.f) : mk(0.5f * w * v.x, 0.5f * w * v.y);
  }
  cx<float> Z[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const cx<float> a = k < UMAX ? H[k] : mk(0.f, 0.f);
    const cx<float> b = (k > 0 && 32 - k < UMAX) ? conj(H[32 - k]) : mk(0.f, 0.f);
    const cx<float> e = a + b;
    const cx<float> o = twiddle_const<64, +1, float>(a - b, k);
    Z[k] = mk(e.re - o.im, e.im + o.re);
  }
  dft<32, +1, float>(Z);
  float best = -INFINITY;
  int bi = 0;
#pragma unroll
  for (int n = 0; n < 32; ++n) {
    // m = 2n then 2n + 1, in increasing m: the first maximum wins
    if (Z[n].re > best) {
      best = Z[n].re;
      bi = 2 * n;
    }
    if (Z[n].im > best) {
      best = Z[n].im;
      bi = 2 * n + 1;
    }
  }
  const long long yy = p / nx, xx = p - yy * nx;
  score[yy * ldOut + xx] = best;
  index[yy * ldOut + xx] = bi;
}

// One wave per group of 16 pixels (grid-stride over groups). C^T = D (A_mat, M = angles)
// times g (B_mat, N = pixels): lane l holds D rows 16 mt + l%16, columns 16 s + 4 (l/16)
// .. + 3, and g of pixel l%16, entries 16 s + 4 (l/16) .. + 3; the result C^T[16 mt +
// 4 (l/16) + j][l%16] comes back in lane l.
template <bool BF16, int MT, int KS>
__global__ void __launch_bounds__(256) k_match_angles_mfma(const float2* __restrict__ stack, int U,
                                                           long long npix, long long pitch, int A,
                                                          const float* __restrict__ dtab,
                                                           float* __restrict__ score, int* __restrict__ index,
                                                           int ldOut, int nx) {
  using SP = Split<BF16>;
  typedef typename SP::T OT;
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lq = l >> 4;
  OT dh[MT][KS], dl[MT][KS];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = dtab[(16 * mt + lr) * 64 + 16 * s + 4 * lq + j];
      SP::split(v, dh[mt][s], dl[mt][s]);
    }
  const long long ngroups = (npix + 15) / 16;
  const long long wstep = (long long)gridDim.x * (blockDim.x >> 6);
  for (long long grp = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); grp < ngroups;
       grp += wstep) {
    const long long p = grp * 16 + lr;
    float v[KS][4];
    float mx = 0.f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int c = 8 * s + 2 * lq;   // entries 2c .. 2c + 3 = components c and c + 1
      const float2 q0 = (p < npix && c < U) ? stack[c * pitch + p] : make_float2(0.f, 0.f);
      const float2 q1 = (p < npix && c + 1 < U) ? stack[(c + 1) * pitch + p] : make_float2(0.f, 0.f);
      v[s][0] = q0.x;
      v[s][1] = q0.y;
      v[s][2] = q1.x;
      v[s][3] = q1.y;
#pragma unroll
      for (int j = 0; j < 4; ++j) mx = fmaxf(mx, fabsf(v[s][j]));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    int ex = 0;
    (void)frexpf(mx, &ex);
    const float f = mx > 0.f ? ldexpf(1.f, 11 - ex) : 1.f;   // mx * f in [2^10, 2^11)
    OT gh[KS], gl[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      float w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) w[j] = v[s][j] * f;
      SP::split(w, gh[s], gl[s]);
    }
    float best = -INFINITY;
    int bi = 0;
    const float inv = 1.f / f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        acc = SP::mma(dh[mt][s], gh[s], acc);
        acc = SP::mma(dh[mt][s], gl[s], acc);
        acc = SP::mma(dl[mt][s], gh[s], acc);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = 16 * mt + 4 * lq + j;
        const float c = acc[j] * inv;
        if (m < A && c > best) {
          best = c;
          bi = m;
        }
      }
    }
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
      const float ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lq == 0 && p < npix) {
      const long long y = p / nx, x = p - y * nx;
      score[y * ldOut + x] = best;
      index[y * ldOut + x] = bi;
    }
  }
}

}  // namespace

hipError_t launch_match_angles(hipStream_t s, int prec, const float* stackf, int U, long long npix, int A,
                               const float* dtab, float* score, int* index, int ldOut, int nx) {
  if (U < 1 || 2 * U > 64 || A < 1 || A > 64 || npix < 1) return hipErrorInvalidValue;
  const float2* stack = reinterpret_cast<const float2*>(stackf);
  const long long pitch = stack_pitch(npix);
  if (prec == 0) {
    const unsigned grid = (unsigned)((npix + 255) / 256);
    if (A == 64) {
#define ECC_MD(UM)                                                                                         \
  hipLaunchKernelGGL((k_match_angles_f32_dft64<UM>), dim3(grid), dim3(256), 0, s, stack, U, npix, pitch, dtab,    \
                     score, index, ldOut, nx)
      if (U <= 8) ECC_MD(8);
      else if (U <= 16) ECC_MD(16);
      else if (U <= 20) ECC_MD(20);
      else if (U <= 24) ECC_MD(24);
      else ECC_MD(32);
#undef ECC_MD
      return last();
    }
#define ECC_MF(UM)                                                                                         \
  hipLaunchKernelGGL((k_match_angles_f32<UM>), dim3(grid), dim3(256), 0, s, stack, U, npix, pitch, A, dtab,      \
                     score, index, ldOut, nx)
    if (U <= 4) ECC_MF(4);
    else if (U <= 8) ECC_MF(8);
    else if (U <= 12) ECC_MF(12);
    else if (U <= 16) ECC_MF(16);
    else if (U <= 18) ECC_MF(18);
    else if (U <= 24) ECC_MF(24);
    else ECC_MF(32);
#undef ECC_MF
    return last();
  }
  if (prec != 1 && prec != 2) return hipErrorInvalidValue;
  const int MT = (A + 15) / 16, KS = (2 * U + 15) / 16;
  const long long groups = (npix + 15) / 16;
  const unsigned grid = (unsigned)std::min<long long>((groups + 3) / 4, 256LL * 8);
#define ECC_MM(BF, mt, ks)                                                                                    \
  if (MT == mt && KS == ks) {                                                                                 \
    hipLaunchKernelGGL((k_match_angles_mfma<BF, mt, ks>), dim3(grid), dim3(256), 0, s, stack, U, npix, pitch, A, \
                       dtab, score, index, ldOut, nx);                                                        \
    return last();                                                                                            \
  }
#define ECC_MM_KS(BF, mt) ECC_MM(BF, mt, 1) ECC_MM(BF, mt, 2) ECC_MM(BF, mt, 3) ECC_MM(BF, mt, 4)
  if (prec == 1) {
    ECC_MM_KS(false, 1) ECC_MM_KS(false, 2) ECC_MM_KS(false, 3) ECC_MM_KS(false, 4)
  } else {
    ECC_MM_KS(true, 1) ECC_MM_KS(true, 2) ECC_MM_KS(true, 3) ECC_MM_KS(true, 4)
  }
#undef ECC_MM_KS
#undef ECC_MM
  return hipErrorInvalidValue;
}

}  // namespace ecc
