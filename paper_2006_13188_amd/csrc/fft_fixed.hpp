// Transforms of compile-time length P = R0 * R1 * R2 (R2 may be 1), one butterfly per
// thread per pass.
//
// This is the self-sorting Stockham recursion with compile-time radices. Pass p has
// radix R_p at stage Ls_p = R_0 * ... * R_{p-1}: butterfly b < P / R_p takes
// in[b + r * P/R_p], multiplies the r-th input by w^{r * (b mod Ls_p)} with
// w = exp(dir 2 pi i / (Ls_p R_p)), and writes its DFT_{R_p} to
// out[(b - j) * R_p + j + r * Ls_p] (j = b mod Ls_p). The first pass takes its inputs
// from the caller's registers and the last pass returns its outputs in registers at
// X[b + r * P/R_last] (natural order), so a transform costs one LDS exchange per pass
// boundary. Intermediate results alternate between two LDS buffers, so each pass
// boundary needs a single barrier. Twiddles come from float64-generated tables.
#pragma once
#include "fft_device.hpp"

namespace ecc {

template <int R0_, int R1_, int R2_>
struct Fixed3 {
  static constexpr int R0 = R0_, R1 = R1_, R2 = R2_;
  static constexpr int P = R0 * R1 * R2;
  static constexpr int N0 = P / R0, N1 = P / R1, N2 = P / R2;   // butterflies per pass
  static constexpr int NT = N0 > N1 ? (N0 > N2 ? N0 : N2) : (N1 > N2 ? N1 : N2);
  static constexpr int TW1 = R0 * (R1 - 1);                       // pass-1 twiddles
  static constexpr int TW2 = (R2 > 1) ? R0 * R1 * (R2 - 1) : 0;   // pass-2 twiddles
  static constexpr int TW = TW1 + TW2;
  static constexpr int RL = (R2 > 1) ? R2 : R1;   // radix of the last pass
  static constexpr int NL = P / RL;                // stride of the last pass outputs
};

// Applies w^{r*j} (table row j, entries r = 1..R-1) to v[1..R-1].
template <int R, int DIR, typename T>
__device__ __forceinline__ void fixed_twiddle(cx<T>* v, const cx<T>* row) {
#pragma unroll
  for (int r = 1; r < R; ++r) v[r] = (DIR < 0) ? cmul(v[r], row[r - 1]) : cmulc(v[r], row[r - 1]);
}

// Pass 0: v holds in[b + r*N0]; writes out[b*R0 + r] to A (element stride ES, offset c).
template <class F, int DIR, int ES, typename T>
__device__ __forceinline__ void fixed_pass0(cx<T>* v, cx<T>* A, int b, int c) {
  dft<F::R0, DIR, T>(v);
#pragma unroll
  for (int r = 0; r < F::R0; ++r) A[(b * F::R0 + r) * ES + c] = v[r];
}

// Pass 1 (Ls = R0): reads A, writes B when R2 > 1; when R2 == 1 it is the last pass and
// leaves X[b + r*N1] in v (v has room for F::RL values).
template <class F, int DIR, int ES, typename T>
__device__ __forceinline__ void fixed_pass1(cx<T>* v, const cx<T>* A, cx<T>* B, const cx<T>* tw, int b, int c) {
#pragma unroll
  for (int r = 0; r < F::R1; ++r) v[r] = A[(b + r * F::N1) * ES + c];
  const int j = b % F::R0;
  if (j != 0) fixed_twiddle<F::R1, DIR, T>(v, tw + j * (F::R1 - 1));
  dft<F::R1, DIR, T>(v);
  if constexpr (F::R2 > 1) {
    const int base = (b - j) * F::R1 + j;
#pragma unroll
    for (int r = 0; r < F::R1; ++r) B[(base + r * F::R0) * ES + c] = v[r];
  }
}

// Pass 2 (Ls = R0*R1, last pass): reads B and leaves X[b + r*N2] in v.
template <class F, int DIR, int ES, typename T>
__device__ __forceinline__ void fixed_pass2(cx<T>* v, const cx<T>* B, const cx<T>* tw, int b, int c) {
#pragma unroll
  for (int r = 0; r < F::R2; ++r) v[r] = B[(b + r * F::N2) * ES + c];
  if (b != 0) fixed_twiddle<F::R2, DIR, T>(v, tw + F::TW1 + b * (F::R2 - 1));
  dft<F::R2, DIR, T>(v);
}

}  // namespace ecc
