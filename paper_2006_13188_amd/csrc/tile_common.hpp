// Building blocks of the on-chip (overlap-save) block kernels: N-point transforms
// (N = 8 M, M = 8, 12, 16) as two Stockham passes over the lines of an LDS image of
// pitch N + 1, for workgroups of 256 threads.
//   pass 0, radix 8:  line element in[b + M r] -> out[8 b + r]      (b < M)
//   pass 1, radix M:  in[b + 8 r] * w^{r b} -> out[b + 8 r]          (b < 8, in place)
// with w = exp(DIR 2 pi i / N); the result is in natural order. Twiddles are compile-time
// tables (float64 values rounded once).
#pragma once
#include "kcommon.hpp"

namespace ecc {
namespace {

constexpr int kTileThreads = 256;


// element pos of line `line` in an LDS image of pitch P: along a row (ROWS) or a column
template <int P, bool ROWS>
__device__ __forceinline__ int at(int line, int pos) {
  return ROWS ? line * P + pos : pos * P + line;
}

// Pass-1 twiddles w^{r b} (w = exp(2 pi i / N), b < 8, r < N/8), float64 rounded once.
template <int N>
struct TileTwiddles {
  float re[8][N / 8], im[8][N / 8];
};
template <int N>
constexpr TileTwiddles<N> make_tile_twiddles() {
  TileTwiddles<N> t{};
  for (int b = 0; b < 8; ++b)
    for (int r = 0; r < N / 8; ++r) {
      t.re[b][r] = (float)cos_turn((long)r * b, N);
      t.im[b][r] = (float)sin_turn((long)r * b, N);
    }
  return t;
}
__constant__ TileTwiddles<64> kTw64 = make_tile_twiddles<64>();
__constant__ TileTwiddles<96> kTw96 = make_tile_twiddles<96>();
__constant__ TileTwiddles<128> kTw128 = make_tile_twiddles<128>();
template <int N>
__device__ __forceinline__ const TileTwiddles<N>& tile_twiddles() {
  if constexpr (N == 64) return kTw64;
  else if constexpr (N == 96) return kTw96;
  else return kTw128;
}

// Pass 0 of the transforms of `nlines` lines of the image in A, all at once: items
// q = t + NT s -> line q mod NL (NL lines per item round), butterfly q / NL.
// Reads everything first, synchronises, then writes (the pass is not in place).
template <int N, int DIR, bool ROWS, int NL, int NT = kTileThreads>
__device__ __forceinline__ void pass0_inplace(cx<float>* A, int t, int nlines, bool act) {
  constexpr int M = N / 8, P = N + 1;
  constexpr int NQ = (NL * M + NT - 1) / NT;
  cx<float> v[NQ][8];
#pragma unroll
  for (int s = 0; s < NQ; ++s) {
    const int q = t + s * NT;
    const int line = q % NL, b = q / NL;
    if (act && b < M && line < nlines) {
#pragma unroll
      for (int r = 0; r < 8; ++r) v[s][r] = A[at<P, ROWS>(line, b + M * r)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NQ; ++s) {
    const int q = t + s * NT;
    const int line = q % NL, b = q / NL;
    if (act && b < M && line < nlines) {
      dft<8, DIR, float>(v[s]);
#pragma unroll
      for (int r = 0; r < 8; ++r) A[at<P, ROWS>(line, 8 * b + r)] = v[s][r];
    }
  }
}

// Pass 1 in place for lines l + LS i (i < NI, line < nlines), butterfly bq (LS = NT / 8
// threads share a butterfly index); tw holds w^{r bq} for the inverse direction
// (conjugated for the forward one).
template <int N, int DIR, bool ROWS, int NI, int NT = kTileThreads>
__device__ __forceinline__ void pass1_inplace(cx<float>* A, const cx<float>* tw, int bq, int l,
                                              int nlines, int nstore) {
  constexpr int M = N / 8, P = N + 1, LS = NT / 8;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int line = l + LS * i;
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

// Loads the N x N window of H (rows y0 - R + i, columns x0 - R + j, zero outside the
// ny x nx image) into the LDS image A as (h, 0), with NT threads, eight loads in flight
// per thread before their LDS stores.
template <int N, int NT>
__device__ __forceinline__ void load_window(cx<float>* A, const float* Hb, int ldH, int ny, int nx, int y0,
                                            int x0, int R, int t) {
  constexpr int P = N + 1, NW = (N * N + NT - 1) / NT, CH = 8;
#pragma unroll 1
  for (int k0 = 0; k0 < NW; k0 += CH) {
    float h[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int q = t + (k0 + k) * NT;
      const int i = q / N, j = q - i * N;
      const int gy = y0 - R + i, gx = x0 - R + j;
      h[k] = 0.f;
      if (q < N * N && gy >= 0 && gy < ny && gx >= 0 && gx < nx) h[k] = Hb[(long long)gy * ldH + gx];
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int q = t + (k0 + k) * NT;
      if (q < N * N) {
        const int i = q / N, j = q - i * N;
        A[i * P + j] = mk(h[k], 0.f);
      }
    }
  }
}

// Forward 2D transform (columns, then rows) of the image in A with NT threads; every
// thread of the workgroup calls it. Ends with a barrier.
template <int N, int NT>
__device__ __forceinline__ void forward_2d(cx<float>* A, int t) {
  constexpr int M = N / 8, LS = NT / 8, NI = (N + LS - 1) / LS;
  const int l = t % LS;
  const int bq = NT == 512 ? __builtin_amdgcn_readfirstlane(t / LS) : t / LS;
  const TileTwiddles<N>& tt = tile_twiddles<N>();
  cx<float> tw[M];
#pragma unroll
  for (int r = 0; r < M; ++r) tw[r] = mk(tt.re[bq][r], tt.im[bq][r]);
  pass0_inplace<N, -1, false, N, NT>(A, t, N, true);
  __syncthreads();
  pass1_inplace<N, -1, false, NI, NT>(A, tw, bq, l, N, N);
  __syncthreads();
  pass0_inplace<N, -1, true, N, NT>(A, t, N, true);
  __syncthreads();
  pass1_inplace<N, -1, true, NI, NT>(A, tw, bq, l, N, N);
  __syncthreads();
}

}  // namespace
}  // namespace ecc
