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


// Workgroup barrier for data exchanged through LDS only: waits for this wave's LDS
// operations (lgkmcnt = 0; vmcnt and expcnt left at their maxima), not for its memory
// loads, so that memory-to-LDS copies can stay in flight across it; the signal fences keep
// the compiler from moving memory accesses across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

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
template <int N, int DIR, bool ROWS, int NL, int NT = kTileThreads, bool LDSB = false>
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
  if constexpr (LDSB) lds_barrier();
  else __syncthreads();
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
// (conjugated for the forward one). Outputs bq + 8 r are stored for r < RS (a bound known
// at compile time, so the others are not computed) and bq + 8 r < nstore.
template <int N, int DIR, bool ROWS, int NI, int NT = kTileThreads, int RS = N / 8>
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
        if (r < RS && bq + 8 * r < nstore) A[at<P, ROWS>(line, bq + 8 * r)] = x[r];
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

// Length-8 DFT of real inputs x (sign DIR): X_0 .. X_7 with X_{8-k} = conj(X_k), from the
// even/odd split of the complex form with the imaginary inputs known to be zero.
template <int DIR>
__device__ __forceinline__ void rdft8(const float* x, cx<float>* X) {
  constexpr float c = float(cos_turn(1, 8)), d = float(DIR);
  const float a0 = x[0] + x[4], a1 = x[0] - x[4], a2 = x[2] + x[6], a3 = x[2] - x[6];
  const float a4 = x[1] + x[5], a5 = x[1] - x[5], a6 = x[3] + x[7], a7 = x[3] - x[7];
  const float e0 = a0 + a2, e2 = a0 - a2, o0 = a4 + a6, o2 = a4 - a6;
  const float dm = a5 - a7, sp = a5 + a7;
  X[0] = mk(e0 + o0, 0.f);
  X[4] = mk(e0 - o0, 0.f);
  X[2] = mk(e2, d * o2);
  X[6] = mk(e2, -d * o2);
  const float r1 = fmadd(c, dm, a1), r3 = fmadd(-c, dm, a1);
  const float i1 = fmadd(c, sp, a3), i3 = fmadd(c, sp, -a3);
  X[1] = mk(r1, d * i1);
  X[7] = mk(r1, -d * i1);
  X[3] = mk(r3, d * i3);
  X[5] = mk(r3, -d * i3);
}

// Forward 2D transform of the block's N x N window of the real signal H (rows
// y0 - R + i, columns x0 - R + j, zero outside the ny x nx image) into A, every thread
// of the workgroup taking part. Column pass 0 reads the window straight from memory
// (real radix 8, all loads of a thread in flight together); since the window is real,
// S[N - k][l] = conj(S[k][(N - l) mod N]), so only rows k <= N/2 are transformed along
// the rows (window_spectrum supplies the others). Ends with a barrier.
// (rows and columns of H outside [ylo, ny) x [xlo, nx) are taken as zero)
// `during` runs once, after the window loads of the first group are issued and before
// their values are used, so that its work overlaps their latency (it must not touch A).
struct NoHook {
  __device__ void operator()() const {}
};
template <int N, int NT, typename Hook = NoHook>
__device__ __forceinline__ void forward_window(cx<float>* A, const float* Hb, int ldH, int ny, int nx, int y0,
                                               int x0, int R, int t, int ylo = 0, int xlo = 0,
                                               Hook during = Hook()) {
  constexpr int M = N / 8, P = N + 1, LS = NT / 8, NI = (N + LS - 1) / LS, H2 = N / 2 + 1;
  constexpr int NQ = (N * M + NT - 1) / NT;   // column pass-0 items of a thread
  constexpr int G = NQ < 4 ? NQ : 4;          // items whose loads are in flight together
  const int l = t % LS;
  const int bq = NT == 512 ? __builtin_amdgcn_readfirstlane(t / LS) : t / LS;
#pragma unroll
  for (int s0 = 0; s0 < NQ; s0 += G) {
    float h[G][8];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int q = t + (s0 + g) * NT;
      const int v = q % N, b = q / N;
      const int gx = x0 - R + v;
      const bool colok = s0 + g < NQ && b < M && gx >= xlo && gx < nx;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int gy = y0 - R + b + M * r;
        h[g][r] = (colok && gy >= ylo && gy < ny) ? Hb[(long long)gy * ldH + gx] : 0.f;
      }
    }
    if (s0 == 0) during();
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int q = t + (s0 + g) * NT;
      const int v = q % N, b = q / N;
      if (s0 + g < NQ && b < M) {
        cx<float> X[8];
        rdft8<-1>(h[g], X);
#pragma unroll
        for (int r = 0; r < 8; ++r) A[(8 * b + r) * P + v] = X[r];
      }
    }
  }
  const TileTwiddles<N>& tt = tile_twiddles<N>();
  cx<float> tw[M];
#pragma unroll
  for (int r = 0; r < M; ++r) tw[r] = mk(tt.re[bq][r], tt.im[bq][r]);
  __syncthreads();
  pass1_inplace<N, -1, false, NI, NT, (H2 + 7) / 8>(A, tw, bq, l, N, H2);
  __syncthreads();
  pass0_inplace<N, -1, true, H2, NT>(A, t, H2, true);
  __syncthreads();
  pass1_inplace<N, -1, true, NI, NT>(A, tw, bq, l, H2, N);
  __syncthreads();
}

// exp(2 pi i m / N), m < N, float64 values rounded once
template <int N>
struct TilePhases {
  float re[N], im[N];
};
template <int N>
constexpr TilePhases<N> make_tile_phases() {
  TilePhases<N> t{};
  for (int m = 0; m < N; ++m) {
    t.re[m] = (float)cos_turn(m, N);
    t.im[m] = (float)sin_turn(m, N);
  }
  return t;
}
__constant__ TilePhases<64> kPh64 = make_tile_phases<64>();
__constant__ TilePhases<96> kPh96 = make_tile_phases<96>();
__constant__ TilePhases<128> kPh128 = make_tile_phases<128>();
template <int N>
__device__ __forceinline__ const TilePhases<N>& tile_phases() {
  if constexpr (N == 64) return kPh64;
  else if constexpr (N == 96) return kPh96;
  else return kPh128;
}

// Spectrum value S[k][v] of a window transformed by forward_window.
template <int N>
__device__ __forceinline__ cx<float> window_spectrum(const cx<float>* A, int k, int v) {
  constexpr int P = N + 1;
  const bool up = k > N / 2;
  const int row = up ? N - k : k;
  const int col = (up && v != 0) ? N - v : v;
  const cx<float> s = A[row * P + col];
  return mk(s.re, up ? -s.im : s.im);
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
