// Tiled (overlap-save) extended correlation: every workgroup owns one T x T block of
// output pixels and keeps the whole computation for it on chip.
//
// The block's N x N input window (rows y0 - R .. y0 - R + N - 1, same for columns; zero
// outside the image) is transformed once. For each component c the product
// hhat * conj(fhat_c) is transformed back, and since the filter spectrum fhat_c belongs to
// F_c placed at window offset (R, R) -> (0, 0) .. (2R, 2R), circular index (u, x) of the
// result equals the linear correlation (H star F_c)(y0 + u, x0 + x) for u, x < N - 2R:
// the cyclic wrap only touches indices past the valid block. The components are then
// combined per pixel with e^{i (kofs + c) alpha(p)} exactly as in the two-pass form
// (section 4, extended correlation by Fourier-domain products), so the only global
// traffic is the signal window, the angle field, the output and the (L2-resident)
// filter spectra.
//
// Transforms have length N = 8 * M (M = 8, 12, 16), done as two Stockham passes:
// pass 0 radix 8 (M butterflies per line, in[b + M r] -> out[8 b + r]), pass 1 radix M
// (8 butterflies per line, in[b + 8 r] -> out[b + 8 r] after the twiddle w^{r b}, so the
// last pass works in place). A 2D transform is a column pass pair then a row pass pair
// on an LDS image of N rows with an odd pitch (conflict-free both along rows and
// columns). Only the T valid rows are carried from the column to the row transforms.
#include "kcommon.hpp"

namespace ecc {

namespace {

constexpr int kTileThreads = 256;

struct TileArgs {
  const float* H;
  long long planeH;
  int ldH;
  Field fld;
  float* y;
  long long planeY;
  int ldY;
  int ny, nx, R, T, tx, ty, U, kofs;
  const float* w;
  float scale;
  const cx<float>* Fs;   // U spectra of N x N
};

// element pos of line `line` in an LDS image of pitch P: along a row (ROWS) or a column
template <int P, bool ROWS>
__device__ __forceinline__ int at(int line, int pos) {
  return ROWS ? line * P + pos : pos * P + line;
}

// Pass 0 of the transforms of `nlines` lines of the image in A, all at once: items
// q = tid + 256 s -> line q mod NL (NL lines per item round), butterfly q / NL.
// Reads everything first, synchronises, then writes (the pass is not in place).
template <int N, int DIR, bool ROWS, int NL>
__device__ __forceinline__ void pass0_inplace(cx<float>* A, int nlines) {
  constexpr int M = N / 8, P = N + 1;
  constexpr int NQ = (NL * M + kTileThreads - 1) / kTileThreads;
  cx<float> v[NQ][8];
#pragma unroll
  for (int s = 0; s < NQ; ++s) {
    const int q = threadIdx.x + s * kTileThreads;
    const int line = q % NL, b = q / NL;
    if (b < M && line < nlines) {
#pragma unroll
      for (int r = 0; r < 8; ++r) v[s][r] = A[at<P, ROWS>(line, b + M * r)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NQ; ++s) {
    const int q = threadIdx.x + s * kTileThreads;
    const int line = q % NL, b = q / NL;
    if (b < M && line < nlines) {
      dft<8, DIR, float>(v[s]);
#pragma unroll
      for (int r = 0; r < 8; ++r) A[at<P, ROWS>(line, 8 * b + r)] = v[s][r];
    }
  }
}

// Pass 1 in place for lines l + 32 i (i < NI, line < nlines), butterfly bq; tw holds
// w^{r bq} for the inverse direction (conjugated for the forward one).
template <int N, int DIR, bool ROWS, int NI>
__device__ __forceinline__ void pass1_inplace(cx<float>* A, const cx<float>* tw, int bq, int l,
                                              int nlines, int nstore) {
  constexpr int M = N / 8, P = N + 1;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int line = l + 32 * i;
    if (line < nlines) {
      cx<float> x[M];
#pragma unroll
      for (int r = 0; r < M; ++r) x[r] = A[at<P, ROWS>(line, bq + 8 * r)];
#pragma unroll
      for (int r = 1; r < M; ++r) x[r] = (DIR > 0) ? cmul(x[r], tw[r]) : cmulc(x[r], tw[r]);
      dft<M, DIR, float>(x);
#pragma unroll
      for (int r = 0; r < M; ++r)
        if (bq + 8 * r < nstore) A[at<P, ROWS>(line, bq + 8 * r)] = x[r];
    }
  }
}

// N: transform length; TV: largest valid block side (a multiple of 32); SEPB: the row
// pass-0 output goes to a second buffer of TV rows (else in place, one more barrier).
template <int N, int TV, bool SEPB>
__global__ void __launch_bounds__(kTileThreads) k_tile_corr(TileArgs a) {
  constexpr int M = N / 8, P = N + 1;
  constexpr int NQ0 = (N * M + kTileThreads - 1) / kTileThreads;   // column pass-0 items
  constexpr int NQ2 = (TV * M + kTileThreads - 1) / kTileThreads;  // row pass-0 items
  constexpr int TR = TV / 32, RV = TV / 8;
  extern __shared__ cx<float> lds_t[];
  cx<float>* A = lds_t;
  cx<float>* Bb = SEPB ? lds_t + N * P : lds_t;
  const int t = threadIdx.x, bq = t >> 5, l = t & 31;
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  const int ntile = a.tx * a.ty;
  const int img = lb / ntile, tile = lb - img * ntile;
  const int y0 = (tile / a.tx) * a.T, x0 = (tile % a.tx) * a.T;
  const int T = a.T;

  // pass-1 twiddles w^{r bq}, w = exp(2 pi i / N), rounded from float64
  cx<float> tw[M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    double sn, cs;
    sincospi(2.0 * (double)(r * bq) / (double)N, &sn, &cs);
    tw[r] = mk((float)cs, (float)sn);
  }

  // ---- signal window into A (real part), zero outside the image
  const float* Hb = a.H + (long long)img * a.planeH;
  for (int q = t; q < N * N; q += kTileThreads) {
    const int i = q / N, j = q - (q / N) * N;
    const int gy = y0 - a.R + i, gx = x0 - a.R + j;
    float h = 0.f;
    if (gy >= 0 && gy < a.ny && gx >= 0 && gx < a.nx) h = Hb[(long long)gy * a.ldH + gx];
    A[i * P + j] = mk(h, 0.f);
  }
  __syncthreads();
  // ---- forward 2D transform of the window: columns, then rows
  pass0_inplace<N, -1, false, N>(A, N);
  __syncthreads();
  pass1_inplace<N, -1, false, N / 32>(A, tw, bq, l, N, N);
  __syncthreads();
  pass0_inplace<N, -1, true, N>(A, N);
  __syncthreads();
  pass1_inplace<N, -1, true, N / 32>(A, tw, bq, l, N, N);
  __syncthreads();
  // signal spectrum values of this thread's column pass-0 items, kept for all components
  cx<float> hs[NQ0][8];
#pragma unroll
  for (int s = 0; s < NQ0; ++s) {
    const int q = t + s * kTileThreads;
    const int v = q % N, b = q / N;
#pragma unroll
    for (int r = 0; r < 8; ++r) hs[s][r] = (b < M) ? A[(b + M * r) * P + v] : mk(0.f, 0.f);
  }

  // ---- per-pixel state of the row pass-1 outputs: pixel (l + 32 i, bq + 8 r)
  float acc[TR][RV];
  cx<float> z[TR][RV], e1[TR][RV];
#pragma unroll
  for (int i = 0; i < TR; ++i) {
#pragma unroll
    for (int r = 0; r < RV; ++r) {
      acc[i][r] = 0.f;
      z[i][r] = mk(0.f, 0.f);
      e1[i][r] = mk(0.f, 0.f);
      const int u = l + 32 * i, x = bq + 8 * r;
      const int gy = y0 + u, gx = x0 + x;
      if (u < T && x < T && gy < a.ny && gx < a.nx) {
        const double al = field_angle(a.fld, a.fld.ptr[(long long)img * a.fld.plane + (long long)gy * a.fld.ld + gx]);
        double sn, cs;
        sincos(al, &sn, &cs);
        e1[i][r] = mk((float)cs, (float)sn);
        sincos((double)a.kofs * al, &sn, &cs);
        z[i][r] = mk((float)cs, (float)sn);
      }
    }
  }

  // filter spectrum values of the first component
  cx<float> fs[NQ0][8];
#pragma unroll
  for (int s = 0; s < NQ0; ++s) {
    const int q = t + s * kTileThreads;
    const int v = q % N, b = q / N;
#pragma unroll
    for (int r = 0; r < 8; ++r) fs[s][r] = (b < M) ? a.Fs[(b + M * r) * N + v] : mk(0.f, 0.f);
  }
  __syncthreads();   // A is rewritten below

  for (int c = 0; c < a.U; ++c) {
    // ---- column pass 0: product, inverse radix 8, A[8 b + r][v]
    const cx<float>* Fn = a.Fs + (long long)(c + 1) * N * N;
    const bool more = c + 1 < a.U;
#pragma unroll
    for (int s = 0; s < NQ0; ++s) {
      const int q = t + s * kTileThreads;
      const int v = q % N, b = q / N;
      if (b < M) {
        cx<float> x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = cmulc(hs[s][r], fs[s][r]);
        if (more) {
#pragma unroll
          for (int r = 0; r < 8; ++r) fs[s][r] = Fn[(b + M * r) * N + v];   // next component
        }
        dft<8, +1, float>(x);
#pragma unroll
        for (int r = 0; r < 8; ++r) A[(8 * b + r) * P + v] = x[r];
      }
    }
    __syncthreads();
    // ---- column pass 1 (in place), rows < T kept
    pass1_inplace<N, +1, false, N / 32>(A, tw, bq, l, N, T);
    __syncthreads();
    // ---- row pass 0 over the T valid rows
    if constexpr (SEPB) {
#pragma unroll
      for (int s = 0; s < NQ2; ++s) {
        const int q = t + s * kTileThreads;
        const int u = q % TV, b = q / TV;
        if (b < M && u < T) {
          cx<float> x[8];
#pragma unroll
          for (int r = 0; r < 8; ++r) x[r] = A[u * P + b + M * r];
          dft<8, +1, float>(x);
#pragma unroll
          for (int r = 0; r < 8; ++r) Bb[u * P + 8 * b + r] = x[r];
        }
      }
    } else {
      pass0_inplace<N, +1, true, TV>(A, T);
    }
    __syncthreads();
    // ---- row pass 1 and the per-pixel combination
    const float wc = a.w[c];
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const int u = l + 32 * i;
      if (u < T) {
        cx<float> x[M];
#pragma unroll
        for (int r = 0; r < M; ++r) x[r] = Bb[u * P + bq + 8 * r];
#pragma unroll
        for (int r = 1; r < M; ++r) x[r] = cmul(x[r], tw[r]);
        dft<M, +1, float>(x);
#pragma unroll
        for (int r = 0; r < RV; ++r) {
          acc[i][r] += wc * (z[i][r].re * x[r].re - z[i][r].im * x[r].im);
          z[i][r] = cmul(z[i][r], e1[i][r]);
        }
      }
    }
    if constexpr (!SEPB) __syncthreads();   // A is rewritten by the next column pass
  }

  float* yb = a.y + (long long)img * a.planeY;
#pragma unroll
  for (int i = 0; i < TR; ++i) {
#pragma unroll
    for (int r = 0; r < RV; ++r) {
      const int u = l + 32 * i, x = bq + 8 * r;
      const int gy = y0 + u, gx = x0 + x;
      if (u < T && x < T && gy < a.ny && gx < a.nx) yb[(long long)gy * a.ldY + gx] = acc[i][r] * a.scale;
    }
  }
}

template <int N, int TV, bool SEPB>
constexpr size_t tile_lds() {
  return (size_t)(SEPB ? N + TV : N) * (N + 1) * sizeof(cx<float>);
}

}  // namespace

#define ECC_TILE_CONFIGS(X) X(64, 64, true) X(96, 64, true) X(128, 64, false) X(128, 96, false)

bool tile_supported(int N, int TV) {
#define ECC_TS(n, tv, sb) if (N == n && TV == tv) return true;
  ECC_TILE_CONFIGS(ECC_TS)
#undef ECC_TS
  return false;
}

size_t tile_lds_bytes(int N, int TV) {
#define ECC_TB(n, tv, sb) if (N == n && TV == tv) return tile_lds<n, tv, sb>();
  ECC_TILE_CONFIGS(ECC_TB)
#undef ECC_TB
  return 0;
}

hipError_t launch_tile_corr(hipStream_t s, int N, int TV, int batch, const float* H, long long planeH,
                            int ldH, const Field& fld, float* y, long long planeY, int ldY, int ny,
                            int nx, int R, int T, int U, int kofs, const float* w, float scale,
                            const cx<float>* Fs) {
  if (T < 1 || T > TV || T > N - 2 * R) return hipErrorInvalidValue;
  TileArgs a;
  a.H = H;
  a.planeH = planeH;
  a.ldH = ldH;
  a.fld = fld;
  a.y = y;
  a.planeY = planeY;
  a.ldY = ldY;
  a.ny = ny;
  a.nx = nx;
  a.R = R;
  a.T = T;
  a.tx = (nx + T - 1) / T;
  a.ty = (ny + T - 1) / T;
  a.U = U;
  a.kofs = kofs;
  a.w = w;
  a.scale = scale;
  a.Fs = Fs;
  const long long nblk = (long long)a.tx * a.ty * batch;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
#define ECC_TL(n, tv, sb)                                                                      \
  if (N == n && TV == tv) {                                                                   \
    hipLaunchKernelGGL((k_tile_corr<n, tv, sb>), dim3((unsigned)nblk), dim3(kTileThreads),    \
                       (tile_lds<n, tv, sb>()), s, a);                                           \
    return last();                                                                             \
  }
  ECC_TILE_CONFIGS(ECC_TL)
#undef ECC_TL
  return hipErrorInvalidValue;
}

hipError_t prepare_tile_kernels() {
  hipError_t e = hipSuccess;
#define ECC_TP(n, tv, sb) \
  if (e == hipSuccess) e = allow_lds(k_tile_corr<n, tv, sb>);
  ECC_TILE_CONFIGS(ECC_TP)
#undef ECC_TP
  return e;
}

}  // namespace ecc
