// Shared device helpers and launch macros of the libecc kernel files.
#pragma once
#include "kernels.hpp"

namespace ecc {

static __device__ __forceinline__ int lds_tw_pad(int n) { return (n + 1) & ~1; }

// XCD-aware block order. The hardware hands workgroup i to XCD (i mod 8); logical
// blocks are dealt so that every XCD receives one contiguous range, and neighbouring
// column tiles (which share 128-byte lines) meet in the same L2. Bijective on [0, n).
static __device__ __forceinline__ int xcd_logical(int bid, int n) {
  const int q = n >> 3, r = n & 7;
  const int xcd = bid & 7, idx = bid >> 3;
  return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// ---------------------------------------------------------------------------------
// Component stacks T_k (ny rows of Px complex values, the inverse column transforms of
// one component) are stored as two planes of ny x ldT: the direct columns v < W and the
// mirror columns Px - v, the latter kept at index v so that both planes are written in
// the same aligned tiles. Element p of row i:
__device__ __forceinline__ cx<float> stack_load(const cx<float>* Tk, int i, int p, int ldT, int ny, int W,
                                                int Px) {
  return p < W ? Tk[i * ldT + p] : Tk[(long long)ny * ldT + i * ldT + (Px - p)];
}

// ---------------------------------------------------------------------------------
// per-pixel phase helpers (float64 recurrence, rounded when used)
struct Phase {
  double re, im;
};
__device__ __forceinline__ Phase pmul(Phase a, Phase b) {
  Phase r;
  r.re = a.re * b.re - a.im * b.im;
  r.im = a.re * b.im + a.im * b.re;
  return r;
}
__device__ __forceinline__ double field_angle(const Field& f, float v) {
  const double x = f.log_mode ? log((double)v) : (double)v;
  return f.mul * x + f.add;
}



#define ECC_NB_SWITCH(NBV, ...)                         \
  switch (NBV) {                                        \
    case 1: { constexpr int NB = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int NB = 2; __VA_ARGS__; } break; \
    case 4: { constexpr int NB = 4; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;               \
  }
#define ECC_EPX_SWITCH(EV, ...)                          \
  switch (EV) {                                          \
    case 1: { constexpr int EPX = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int EPX = 2; __VA_ARGS__; } break; \
    case 4: { constexpr int EPX = 4; __VA_ARGS__; } break; \
    case 8: { constexpr int EPX = 8; __VA_ARGS__; } break; \
    case 16: { constexpr int EPX = 16; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                \
  }
#define ECC_EPP_SWITCH(EV, ...)                          \
  switch (EV) {                                          \
    case 1: { constexpr int EPP = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int EPP = 2; __VA_ARGS__; } break; \
    case 4: { constexpr int EPP = 4; __VA_ARGS__; } break; \
    case 8: { constexpr int EPP = 8; __VA_ARGS__; } break; \
    case 16: { constexpr int EPP = 16; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                \
  }
#define ECC_EPC_SWITCH(EV, ...)                          \
  switch (EV) {                                          \
    case 4: { constexpr int EPT = 4; __VA_ARGS__; } break; \
    case 5: { constexpr int EPT = 5; __VA_ARGS__; } break; \
    case 6: { constexpr int EPT = 6; __VA_ARGS__; } break; \
    case 8: { constexpr int EPT = 8; __VA_ARGS__; } break; \
    case 9: { constexpr int EPT = 9; __VA_ARGS__; } break; \
    case 12: { constexpr int EPT = 12; __VA_ARGS__; } break; \
    case 16: { constexpr int EPT = 16; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                \
  }
#define ECC_NB12_SWITCH(NBV, ...)                        \
  switch (NBV) {                                        \
    case 1: { constexpr int NB = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int NB = 2; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;               \
  }
#define ECC_EPT_SWITCH(EV, ...)                          \
  switch (EV) {                                          \
    case 4: { constexpr int EPT = 4; __VA_ARGS__; } break; \
    case 8: { constexpr int EPT = 8; __VA_ARGS__; } break; \
    case 12: { constexpr int EPT = 12; __VA_ARGS__; } break; \
    case 16: { constexpr int EPT = 16; __VA_ARGS__; } break; \
    case 24: { constexpr int EPT = 24; __VA_ARGS__; } break; \
    case 32: { constexpr int EPT = 32; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                \
  }

static inline hipError_t last() { return hipGetLastError(); }

template <typename K>
static hipError_t allow_lds(K kernel) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

}  // namespace ecc
