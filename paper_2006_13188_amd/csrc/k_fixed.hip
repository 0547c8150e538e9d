// Correlation kernels specialised for transform lengths with a compiled three-pass
// schedule P = R0 * R1 * R2 (see fft_fixed.hpp). Same results as the LDS-engine
// kernels in k_corr.hip with compile-time indexing and one barrier per pass boundary.
#include "fft_fixed.hpp"
#include "kcommon.hpp"

namespace ecc {

// Column kernel: a tile of B adjacent source columns v and components [k0, k1). The
// direct column v and the mirror column Px - v of every component are transformed
// together: 2B transforms share one LDS buffer (slot c < B: direct, slot B + c:
// mirror), updated in place (each pass reads its inputs into registers, synchronises,
// then writes). The signal spectrum of the tile stays in registers for the whole chunk
// and each filter spectrum value is read once. NTH threads share the butterflies of a
// pass: item q has slot q mod 2B and butterfly q / 2B. Products and conj_mode as in
// k_corr_cols (k_corr.hip); the two results go to the direct and mirror planes of T_k.
template <class F, int B, int NTH, bool FULL, int CM>
__global__ void __launch_bounds__(NTH) k_corr_cols_w(
    const cx<float>* __restrict__ Hh, long long planeHh, int ldHh, const cx<float>* __restrict__ Fh,
    long long planeFk, int ldF, const float* __restrict__ parity, cx<float>* __restrict__ T,
    long long planeTk, long long planeTimg, int ldT, int ny, int Px, int W, int U, int kchunk,
    int nxb, int nch, const cx<float>* __restrict__ twg) {
  constexpr int conj_mode = CM;
  constexpr int Py = F::P;
  constexpr int S2 = 2 * B;                      // transform slots
  static_assert(NTH % S2 == 0, "NTH must be a multiple of 2B");
  constexpr int BS = NTH / S2;                   // butterflies per sweep of the threads
  constexpr int I0 = (B * F::N0 + NTH - 1) / NTH;   // pass 0 runs per source column
  constexpr int I1 = (F::N1 + BS - 1) / BS;
  constexpr int I2 = (F::N2 + BS - 1) / BS;
  extern __shared__ cx<float> smem_f[];
  cx<float>* tw = smem_f;
  cx<float>* A = smem_f + ((F::TW + 1) & ~1);
  for (int i = threadIdx.x; i < F::TW; i += NTH) tw[i] = twg[i];
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  const int xb = lb % nxb, rest = lb / nxb;
  const int ch = rest % nch, img = rest / nch;
  const int k0 = ch * kchunk, k1 = min(U, k0 + kchunk);
  const int v0 = xb * B;
  // pass 0: item q = threadIdx.x + it*NTH -> source column c0 = q % B, butterfly q / B
  // passes 1, 2: slot s = threadIdx.x % S2, butterfly threadIdx.x / S2 + it*BS
  const int s = threadIdx.x % S2, bb = threadIdx.x / S2;
  const cx<float>* Hb = Hh + (long long)img * planeHh;
  __syncthreads();
  for (int k = k0; k < k1; ++k) {
    const cx<float>* Fk = Fh + (long long)k * planeFk;
    const float par = FULL ? 1.f : parity[k];
    cx<float>* Tk = T + (long long)img * planeTimg + (long long)k * planeTk;
    // ---- pass 0: direct and mirror products from one read of the spectra (the signal
    // spectrum is re-read from L2 for every component), DFT_R0, write A
#pragma unroll 1
    for (int it = 0; it < I0; ++it) {
      const int q = threadIdx.x + it * NTH;
      const int c0 = q % B, b = q / B, v = v0 + c0;
      if (b < F::N0) {
        const bool vin = v < W;
        const int vm = (v == 0) ? 0 : Px - v;
        cx<float> hv[F::R0], ga[F::R0];
#pragma unroll
        for (int r = 0; r < F::R0; ++r) {
          const int u = b + r * F::N0;
          hv[r] = mk(0.f, 0.f);
          ga[r] = mk(0.f, 0.f);
          if (vin) {
            hv[r] = Hb[u * ldHh + v];
            ga[r] = Fk[u * ldF + v];
          }
        }
        cx<float> x[F::R0];
        // direct slot: conj_mode 0: h conj a; 1: h a; 2: h b
#pragma unroll
        for (int r = 0; r < F::R0; ++r) {
          if constexpr (conj_mode == 2) {
            const int u = b + r * F::N0;
            const cx<float> gb = FULL ? (vin ? Fk[((u == 0) ? 0 : Py - u) * ldF + vm] : mk(0.f, 0.f))
                                      : scale(ga[r], par);
            x[r] = cmul(hv[r], gb);
          } else {
            x[r] = conj_mode == 0 ? cmulc(hv[r], ga[r]) : cmul(hv[r], ga[r]);
          }
        }
        dft<F::R0, +1, float>(x);
#pragma unroll
        for (int r = 0; r < F::R0; ++r) A[(b * F::R0 + r) * S2 + c0] = x[r];
        // mirror slot: conj_mode 0: h b; 1: h conj b; 2: h conj a
#pragma unroll
        for (int r = 0; r < F::R0; ++r) {
          if constexpr (conj_mode == 2) {
            x[r] = cmulc(hv[r], ga[r]);
          } else {
            const int u = b + r * F::N0;
            const cx<float> gb = FULL ? (vin ? Fk[((u == 0) ? 0 : Py - u) * ldF + vm] : mk(0.f, 0.f))
                                      : scale(ga[r], par);
            x[r] = conj_mode == 0 ? cmul(hv[r], gb) : cmulc(hv[r], gb);
          }
        }
        dft<F::R0, +1, float>(x);
#pragma unroll
        for (int r = 0; r < F::R0; ++r) A[(b * F::R0 + r) * S2 + B + c0] = x[r];
      }
    }
    __syncthreads();
    // ---- pass 1 (Ls = R0)
    {
      cx<float> y[I1][F::R1];
#pragma unroll
      for (int it = 0; it < I1; ++it) {
        const int b = bb + it * BS;
        if (b < F::N1) {
#pragma unroll
          for (int r = 0; r < F::R1; ++r) y[it][r] = A[(b + r * F::N1) * S2 + s];
        }
      }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < I1; ++it) {
        const int b = bb + it * BS;
        if (b < F::N1) {
          const int j = b % F::R0;
          if (j != 0) fixed_twiddle<F::R1, +1, float>(y[it], tw + j * (F::R1 - 1));
          dft<F::R1, +1, float>(y[it]);
          const int base = (b - j) * F::R1 + j;
#pragma unroll
          for (int r = 0; r < F::R1; ++r) A[(base + r * F::R0) * S2 + s] = y[it][r];
        }
      }
    }
    __syncthreads();
    // ---- pass 2 (Ls = R0 R1, last): outputs X[b + r*N2] to the stack planes
    {
      cx<float> z[I2][F::R2];
#pragma unroll
      for (int it = 0; it < I2; ++it) {
        const int b = bb + it * BS;
        if (b < F::N2) {
#pragma unroll
          for (int r = 0; r < F::R2; ++r) z[it][r] = A[(b + r * F::N2) * S2 + s];
        }
      }
      __syncthreads();   // pass 0 of the next component rewrites A
      const bool mir = s >= B;
      const int v = v0 + (mir ? s - B : s);
      cx<float>* dst = mir ? Tk + (long long)ny * ldT : Tk;
      const bool keep = v < W && (!mir || (v != 0 && 2 * v != Px));
#pragma unroll
      for (int it = 0; it < I2; ++it) {
        const int b = bb + it * BS;
        if (b < F::N2) {
          if (b != 0) fixed_twiddle<F::R2, +1, float>(z[it], tw + F::TW1 + b * (F::R2 - 1));
          dft<F::R2, +1, float>(z[it]);
          if (keep) {
#pragma unroll
            for (int r = 0; r < F::R2; ++r) {
              const int i = b + r * F::N2;
              if (i < ny) dst[i * ldT + v] = mir ? conj(z[it][r]) : z[it][r];
            }
          }
        }
      }
    }
  }
}

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

hipError_t launch_corr_cols_fixed(hipStream_t s, int Bc, int batch, int kchunk, const cx<float>* Hh,
                                  long long planeHh, int ldHh, const cx<float>* Fh, long long planeFk,
                                  int ldF, int fullplane, const float* parity, cx<float>* T,
                                  long long planeTk, long long planeTimg, int ldT, int ny, int Px, int W,
                                  int U, int conj_mode, int Py, const cx<float>* tw) {
  const int nxb = (W + Bc - 1) / Bc, nch = (U + kchunk - 1) / kchunk;
  dim3 grid(nxb * nch * batch);
#define ECC_CCB3(a, b_, c_, BB, NN, FU, CMV)                                                     \
  if (conj_mode == CMV && fullplane == FU)                                                      \
    hipLaunchKernelGGL((k_corr_cols_w<Fixed3<a, b_, c_>, BB, NN, FU, CMV>), grid, dim3(NN), lds, s, Hh, \
                       planeHh, ldHh, Fh, planeFk, ldF, parity, T, planeTk, planeTimg, ldT, ny, Px, \
                       W, U, kchunk, nxb, nch, tw);
#define ECC_CCB(a, b_, c_, BB, NN)                                                                \
  if (Bc == BB) {                                                                               \
    using F = Fixed3<a, b_, c_>;                                                                \
    const size_t lds = sizeof(cx<float>) * (((F::TW + 1) & ~1) + (size_t)F::P * 2 * BB);        \
    if (lds > 160 * 1024) return hipErrorInvalidValue;                                          \
    ECC_CCB3(a, b_, c_, BB, NN, 0, 0) ECC_CCB3(a, b_, c_, BB, NN, 0, 1) ECC_CCB3(a, b_, c_, BB, NN, 0, 2) \
    ECC_CCB3(a, b_, c_, BB, NN, 1, 0) ECC_CCB3(a, b_, c_, BB, NN, 1, 1) ECC_CCB3(a, b_, c_, BB, NN, 1, 2) \
    return hipGetLastError();                                                                   \
  }
#define ECC_CC(a, b_, c_)                      \
  if (Py == (a) * (b_) * (c_)) {               \
    ECC_CCB(a, b_, c_, 4, 512)                 \
    ECC_CCB(a, b_, c_, 8, 1024)                \
    return hipErrorInvalidValue;               \
  }
  ECC_FIXED_SIZES(ECC_CC)
#undef ECC_CC
#undef ECC_CCB
  return hipErrorInvalidValue;
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
#define ECC_PFC(a, b_, c_, BB, NN, FU) ECC_ALLOW(k_corr_cols_w<Fixed3<a, b_, c_>, BB, NN, FU, 0>); \
  ECC_ALLOW(k_corr_cols_w<Fixed3<a, b_, c_>, BB, NN, FU, 1>); ECC_ALLOW(k_corr_cols_w<Fixed3<a, b_, c_>, BB, NN, FU, 2>);
#define ECC_PF(a, b_, c_)                                                                          \
  ECC_PFC(a, b_, c_, 4, 512, true) ECC_PFC(a, b_, c_, 4, 512, false)                               \
  ECC_PFC(a, b_, c_, 8, 1024, true) ECC_PFC(a, b_, c_, 8, 1024, false)                             \
  ECC_ALLOW(k_corr_rows_x<Fixed3<a, b_, c_>, 1>); ECC_ALLOW(k_corr_rows_x<Fixed3<a, b_, c_>, 2>);   \
  ECC_ALLOW(k_corr_rows_x<Fixed3<a, b_, c_>, 4>);
  ECC_FIXED_SIZES(ECC_PF)
#undef ECC_PF
  return e;
}

}  // namespace ecc
