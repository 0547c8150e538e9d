// Row kernel of the two-pass correlation specialised for transform lengths with a
// compiled three-pass schedule P = R0 * R1 * R2 (see fft_fixed.hpp). Same results as the
// LDS-engine row kernel in k_corr.hip with compile-time indexing and one barrier per pass
// boundary.
#include "fft_fixed.hpp"
#include "kcommon.hpp"

namespace ecc {

// Row kernel: NR image rows per workgroup, each row's components transformed one after
// another by its own thread group; pixel x = b + r*NL of the row (r < RL) belongs to
// thread b, which keeps e^{i k alpha(x)} (float64 recurrence) and the sums:
//   y(x) = scale * sum_k w_k Re(e^{i k alpha(x)} G_k(x))   (+ the adjoint's second output)
// The first-pass inputs of component k + 1 are loaded while component k is transformed.
template <class F, int NR>
__global__ void __launch_bounds__(640) k_corr_rows_x(
    const cx<float>* __restrict__ T, long long planeTk, long long planeTimg, int ldT, Field fld,
    float* __restrict__ y, long long planeY, int ldY, int ny, int nx, int U,
    const float* __restrict__ w, float scl, float* __restrict__ y2, const float* __restrict__ mulsig,
    long long planeMul, int ldMul, float y2scale, int kofs, int accum,
    const cx<float>* __restrict__ twg) {
  constexpr int Px = F::P;
  constexpr int RM = F::R0 > F::R1 ? (F::R0 > F::R2 ? F::R0 : F::R2) : (F::R1 > F::R2 ? F::R1 : F::R2);
  extern __shared__ cx<float> smem_f[];
  cx<float>* tw = smem_f;
  for (int i = threadIdx.x; i < F::TW; i += blockDim.x) tw[i] = twg[i];
  const int c = threadIdx.x / F::NT, b = threadIdx.x - c * F::NT;
  const int row = blockIdx.x * NR + c, img = blockIdx.y;
  const bool act = c < NR && row < ny;   // threads past NR * NT (rounding to waves) idle
  cx<float>* A = smem_f + ((F::TW + 1) & ~1) + (2 * (c < NR ? c : 0)) * F::P;
  cx<float>* Bf = A + F::P;
  const bool own = act && b < F::NL;
  Phase z[F::RL], e1[F::RL];
  float acc[F::RL], acc2[F::RL];
#pragma unroll
  for (int r = 0; r < F::RL; ++r) {
    const int x = b + r * F::NL;
    z[r].re = 1.0;
    z[r].im = 0.0;
    e1[r] = z[r];
    acc[r] = 0.f;
    acc2[r] = 0.f;
    if (own && x < nx) {
      const double a = field_angle(fld, fld.ptr[(long long)img * fld.plane + (long long)row * fld.ld + x]);
      double sn, cs;
      sincos(a, &sn, &cs);
      e1[r].re = cs;
      e1[r].im = sn;
      sincos((double)kofs * a, &sn, &cs);   // first component of this launch: kofs
      z[r].re = cs;
      z[r].im = sn;
    }
  }
  const cx<float>* Tb = T + (long long)img * planeTimg;
  const int rr = act ? row : 0;
  constexpr int W = Px / 2 + 1;
  cx<float> xn[F::R0];
  const bool p0 = act && b < F::N0;
  if (p0) {
#pragma unroll
    for (int r = 0; r < F::R0; ++r) xn[r] = stack_load(Tb, rr, b + r * F::N0, ldT, ny, W, Px);
  }
  __syncthreads();
  for (int k = 0; k < U; ++k) {
    cx<float> x[RM];
    if (p0) {
#pragma unroll
      for (int r = 0; r < F::R0; ++r) x[r] = xn[r];
      if (k + 1 < U) {
        const cx<float>* src = Tb + (long long)(k + 1) * planeTk;
#pragma unroll
        for (int r = 0; r < F::R0; ++r) xn[r] = stack_load(src, rr, b + r * F::N0, ldT, ny, W, Px);
      }
      fixed_pass0<F, +1, 1, float>(x, A, b, 0);
    }
    __syncthreads();
    if (act && b < F::N1) fixed_pass1<F, +1, 1, float>(x, A, Bf, tw, b, 0);
    if constexpr (F::R2 > 1) {
      __syncthreads();
      if (act && b < F::N2) fixed_pass2<F, +1, 1, float>(x, Bf, tw, b, 0);
    }
    if (own) {
      const float wk = w[k];
#pragma unroll
      for (int r = 0; r < F::RL; ++r) {
        const float zr = (float)z[r].re, zi = (float)z[r].im;
        acc[r] += wk * (zr * x[r].re - zi * x[r].im);
        if (y2) acc2[r] += wk * (float)(kofs + k) * (zr * x[r].im + zi * x[r].re);
        z[r] = pmul(z[r], e1[r]);
      }
    }
    if constexpr (F::R2 == 1) __syncthreads();
  }
  if (own) {
#pragma unroll
    for (int r = 0; r < F::RL; ++r) {
      const int x = b + r * F::NL;
      if (x < nx) {
        const long long o = (long long)img * planeY + (long long)row * ldY + x;
        y[o] = accum ? y[o] + acc[r] * scl : acc[r] * scl;
        if (y2) {
          const float v2 = acc2[r] * scl * y2scale * mulsig[(long long)img * planeMul + (long long)row * ldMul + x];
          y2[o] = accum ? y2[o] + v2 : v2;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// host side: compiled schedules (P, R0, R1, R2)
#define ECC_FIXED_SIZES(X) X(5, 3, 9) X(7, 15, 5) X(15, 10, 7) X(12, 10, 9)

bool fixed_split(int P, int* R0, int* R1, int* R2) {
#define ECC_FS(a, b, c) if (P == (a) * (b) * (c)) { *R0 = (a); *R1 = (b); *R2 = (c); return true; }
  ECC_FIXED_SIZES(ECC_FS)
#undef ECC_FS
  return false;
}

hipError_t launch_corr_rows_fixed(hipStream_t s, int NR, int batch, const cx<float>* T, long long planeTk,
                                  long long planeTimg, int ldT, const Field& fld, float* y,
                                  long long planeY, int ldY, int ny, int nx, int U, const float* w,
                                  float scale_, float* y2, const float* mulsig, long long planeMul,
                                  int ldMul, float y2scale, int kofs, int accum, int Px,
                                  const cx<float>* tw) {
#define ECC_CRN(a, b_, c_, NN)                                                                   \
  if (NR == NN) {                                                                               \
    using F = Fixed3<a, b_, c_>;                                                                \
    const int nthr = (NN * F::NT + 63) / 64 * 64;                                               \
    if (nthr > 640) return hipErrorInvalidValue;                                                \
    const size_t lds = sizeof(cx<float>) * (((F::TW + 1) & ~1) + 2 * (size_t)F::P * NN);        \
    dim3 grid((ny + NN - 1) / NN, batch);                                                       \
    hipLaunchKernelGGL((k_corr_rows_x<F, NN>), grid, dim3(nthr), lds, s, T, planeTk, planeTimg, ldT, \
                       fld, y, planeY, ldY, ny, nx, U, w, scale_, y2, mulsig, planeMul, ldMul,  \
                       y2scale, kofs, accum, tw);                                               \
    return hipGetLastError();                                                                   \
  }
#define ECC_CR(a, b_, c_)                      \
  if (Px == (a) * (b_) * (c_)) {               \
    ECC_CRN(a, b_, c_, 1)                      \
    ECC_CRN(a, b_, c_, 2)                      \
    ECC_CRN(a, b_, c_, 4)                      \
    return hipErrorInvalidValue;               \
  }
  ECC_FIXED_SIZES(ECC_CR)
#undef ECC_CR
#undef ECC_CRN
  return hipErrorInvalidValue;
}

hipError_t prepare_fixed_kernels() {
  hipError_t e = hipSuccess;
#define ECC_ALLOW(...) if (e == hipSuccess) e = allow_lds(__VA_ARGS__)
#define ECC_PF(a, b_, c_)                                                                          \
  ECC_ALLOW(k_corr_rows_x<Fixed3<a, b_, c_>, 1>); ECC_ALLOW(k_corr_rows_x<Fixed3<a, b_, c_>, 2>);   \
  ECC_ALLOW(k_corr_rows_x<Fixed3<a, b_, c_>, 4>);
  ECC_FIXED_SIZES(ECC_PF)
#undef ECC_PF
#undef ECC_ALLOW
  return e;
}

}  // namespace ecc
