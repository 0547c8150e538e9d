// Device-side FFT engine for gfx950: mixed-radix (2,3,4,5,6,7,8)
// Stockham autosort transforms staged through LDS, with register butterflies.
//
// One workgroup runs B transforms of length P at once. Two layouts are supported:
//   interleaved (column kernels): element `pos` of transform c sits at buf[pos*B + c],
//     so B adjacent image columns map to contiguous LDS words;
//   blocked (row kernels): element `pos` of transform c sits at buf[c*Pst + pos].
// Every pass reads all of a thread's butterfly inputs into registers, synchronises,
// then writes the outputs back in place (one LDS buffer per transform).
//
// A pass with radix R at stage Ls (product of the earlier radices) computes, for
// butterfly b in [0, P/R) with j = b mod Ls:
//   x_r = in[b + r*P/R] * w^{r*j},  w = exp(dir * 2*pi*i / (Ls*R))
//   out[(b - j)*R + j + r*Ls] = DFT_R(x)_r
// which leaves the result in natural order (decimation in time, self-sorting).
// Twiddles come from a table generated in float64 on the host and staged in LDS.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecc {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.re = a; r.im = b; return r; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {  // a * conj(b)
  return mk(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return mk(a.re, -a.im); }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.re * s, a.im * s); }
// i * a * sgn
template <int SGN, typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  if constexpr (SGN > 0) return mk(-a.im, a.re);
  else return mk(a.im, -a.re);
}

// ---------------------------------------------------------------- compile-time trig
// cos / sin of 2*pi*m/n evaluated in double by a Taylor series on [-pi, pi]
// (30 terms: truncation far below double rounding), used for butterfly constants.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int i = 1; i < 30; ++i) {
    term *= -x * x / double((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 30; ++i) {
    term *= -x * x / double((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}
constexpr double reduce_turn(long m, long n) {  // angle of m/n turns in [-pi, pi]
  long r = m % n;
  if (r < 0) r += n;
  if (2 * r > n) r -= n;
  return 2.0 * kPi * double(r) / double(n);
}
constexpr double cos_turn(long m, long n) {
  long r = ((m % n) + n) % n;
  if (4 * r == n || 4 * r == 3 * n) return 0.0;
  if (2 * r == n) return -1.0;
  if (r == 0) return 1.0;
  return taylor_cos(reduce_turn(m, n));
}
constexpr double sin_turn(long m, long n) {
  long r = ((m % n) + n) % n;
  if (r == 0 || 2 * r == n) return 0.0;
  if (4 * r == n) return 1.0;
  if (4 * r == 3 * n) return -1.0;
  return taylor_sin(reduce_turn(m, n));
}

constexpr int smallest_factor(int n) {
  for (int p = 2; p * p <= n; ++p)
    if (n % p == 0) return p;
  return n;
}

// ---------------------------------------------------------------- butterflies
// In-register DFT of length R: v_q <- sum_n v_n exp(DIR * 2*pi*i*n*q/R).
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T>* v);

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_odd_prime(cx<T>* v) {
  constexpr int h = (R - 1) / 2;
  cx<T> a[h + 1], b[h + 1];
#pragma unroll
  for (int n = 1; n <= h; ++n) {
    a[n] = v[n] + v[R - n];
    b[n] = v[n] - v[R - n];
  }
  cx<T> x0 = v[0];
  cx<T> s = x0;
#pragma unroll
  for (int n = 1; n <= h; ++n) s = s + a[n];
  v[0] = s;
#pragma unroll
  for (int q = 1; q <= h; ++q) {
    cx<T> A = x0, B = mk<T>(0, 0);
#pragma unroll
    for (int n = 1; n <= h; ++n) {
      const T c = T(cos_turn(n * q, R));
      const T sn = T(sin_turn(n * q, R));
      A.re += a[n].re * c;
      A.im += a[n].im * c;
      B.re += b[n].re * sn;
      B.im += b[n].im * sn;
    }
    const cx<T> iB = mul_i<DIR>(B);
    v[q] = A + iB;
    v[R - q] = A - iB;
  }
}

// a * exp(DIR 2 pi i m / R); m is a constant once the caller's loops are unrolled, and
// the factors 1, -1 and +-i cost no arithmetic (a product with an exact 0 or 1 would
// still be computed: the compiler may not drop it because of signed zeros).
template <int R, int DIR, typename T>
__device__ __forceinline__ cx<T> twiddle_const(cx<T> a, int m) {
  const int r = ((m % R) + R) % R;
  if (r == 0) return a;
  if (2 * r == R) return mk(-a.re, -a.im);
  if (4 * r == R) return mul_i<DIR>(a);
  if (4 * r == 3 * R) return mul_i<-DIR>(a);
  return cmul(a, mk<T>(T(cos_turn(r, R)), T(DIR * sin_turn(r, R))));
}

// Cooley-Tukey split R = R1 R2: R2 transforms of length R1 over n1 (inputs v[R2 n1 + n2]),
// twiddles, then R1 transforms of length R2.
template <int R1, int R2, int DIR, typename T>
__device__ __forceinline__ void dft_composite(cx<T>* v) {
  constexpr int R = R1 * R2;
  cx<T> y[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
    cx<T> t[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + n2];
    dft<R1, DIR, T>(t);
#pragma unroll
    for (int q1 = 0; q1 < R1; ++q1) y[n2][q1] = twiddle_const<R, DIR, T>(t[q1], n2 * q1);
  }
#pragma unroll
  for (int q1 = 0; q1 < R1; ++q1) {
    cx<T> u[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) u[n2] = y[n2][q1];
    dft<R2, DIR, T>(u);
#pragma unroll
    for (int q2 = 0; q2 < R2; ++q2) v[q1 + R1 * q2] = u[q2];
  }
}

constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }
// inverse of a modulo m (gcd(a, m) = 1, m > 1)
constexpr int inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}
// largest power of a prime dividing R (R itself when R is a prime power)
constexpr int prime_power_part(int R) {
  const int p = smallest_factor(R);
  int q = 1;
  while (R % (q * p) == 0) q *= p;
  return q;
}

// Prime-factor (Good-Thomas) split of R = R1 R2 with gcd(R1, R2) = 1: input index
// (R2 n1 + R1 n2) mod R and output index (R2 (R2^-1 mod R1) q1 + R1 (R1^-1 mod R2) q2)
// mod R (Chinese remainders) turn the transform into plain length-R1 and length-R2
// transforms with no twiddle factors.
template <int R1, int R2, int DIR, typename T>
__device__ __forceinline__ void dft_prime_factor(cx<T>* v) {
  constexpr int R = R1 * R2;
  constexpr int C1 = R2 * inv_mod(R2 % R1, R1), C2 = R1 * inv_mod(R1 % R2, R2);
  cx<T> y[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) y[n2][n1] = v[(R2 * n1 + R1 * n2) % R];
    dft<R1, DIR, T>(y[n2]);
  }
#pragma unroll
  for (int q1 = 0; q1 < R1; ++q1) {
    cx<T> u[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) u[n2] = y[n2][q1];
    dft<R2, DIR, T>(u);
#pragma unroll
    for (int q2 = 0; q2 < R2; ++q2) v[(C1 * q1 + C2 * q2) % R] = u[q2];
  }
}

template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    const cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 3) {
    // with a = v1 + v2, b = v1 - v2: X0 = v0 + a, X1,2 = v0 - a/2 +- DIR i (sqrt(3)/2) b,
    // the last product folded into fused multiply-adds
    constexpr T h = T(-cos_turn(1, 3)), sn = T(DIR * sin_turn(1, 3));
    const cx<T> a = v[1] + v[2], b = v[1] - v[2];
    const cx<T> A = mk(fmadd(-h, a.re, v[0].re), fmadd(-h, a.im, v[0].im));
    v[0] = v[0] + a;
    v[1] = mk(fmadd(-sn, b.im, A.re), fmadd(sn, b.re, A.im));
    v[2] = mk(fmadd(sn, b.im, A.re), fmadd(-sn, b.re, A.im));
  } else if constexpr (R == 8) {
    // radix 2 over two length-4 transforms (even and odd samples): X_k = E_k + W^k O_k,
    // X_{k+4} = E_k - W^k O_k with W = exp(DIR 2 pi i / 8) = c (1 + DIR i), W^2 = DIR i,
    // W^3 = c (-1 + DIR i); the factor c is folded into fused multiply-adds
    cx<T> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft<4, DIR, T>(e);
    dft<4, DIR, T>(o);
    constexpr T c = T(cos_turn(1, 8)), d = T(DIR);
    const T p1 = o[1].re - d * o[1].im, q1 = o[1].im + d * o[1].re;    // W O_1 / c
    const T p3 = -o[3].re - d * o[3].im, q3 = d * o[3].re - o[3].im;   // W^3 O_3 / c
    const cx<T> w2 = mul_i<DIR>(o[2]);
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[2] = e[2] + w2;
    v[6] = e[2] - w2;
    v[1] = mk(fmadd(c, p1, e[1].re), fmadd(c, q1, e[1].im));
    v[5] = mk(fmadd(-c, p1, e[1].re), fmadd(-c, q1, e[1].im));
    v[3] = mk(fmadd(c, p3, e[3].re), fmadd(c, q3, e[3].im));
    v[7] = mk(fmadd(-c, p3, e[3].re), fmadd(-c, q3, e[3].im));
  } else if constexpr (R == 4) {
    const cx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
    const cx<T> s13 = v[1] + v[3], d13 = mul_i<DIR>(v[1] - v[3]);
    v[0] = s02 + s13;
    v[2] = s02 - s13;
    v[1] = d02 + d13;
    v[3] = d02 - d13;
  } else if constexpr (smallest_factor(R) == R) {
    dft_odd_prime<R, DIR, T>(v);
  } else if constexpr (prime_power_part(R) != R) {
    dft_prime_factor<prime_power_part(R), R / prime_power_part(R), DIR, T>(v);
  } else if constexpr (R % 4 == 0 && R != 4) {
    dft_composite<4, R / 4, DIR, T>(v);
  } else {
    dft_composite<smallest_factor(R), R / smallest_factor(R), DIR, T>(v);
  }
}

// ---------------------------------------------------------------- transform descriptor
constexpr int kMaxPass = 8;

struct FftDesc {
  int P;
  int npass;
  int twsize;                 // twiddle table entries (complex)
  int radix[kMaxPass];
  int twoff[kMaxPass];        // offset of each pass's twiddles in the table
  uint32_t magic[kMaxPass];   // floor(2^32 / Ls) + 1 for Ls > 1 (exact for b, Ls < 2^16)
};

struct Layout {
  int B;      // transforms per workgroup
  int lgB;    // log2(B) for the interleaved layout
  int Pst;    // stride between transforms in the blocked layout
};

template <bool ILV>
__device__ __forceinline__ int addr(const Layout& L, int c, int pos) {
  if constexpr (ILV) return (pos << L.lgB) + c;
  else return c * L.Pst + pos;
}

template <int R, int NB, int DIR, bool ILV, typename T>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, const Layout& L, int P, int Ls,
                                              uint32_t magic, const cx<T>* tw, int c, int f,
                                              int TF, bool active) {
  const int nb = P / R;
  cx<T> v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = f + i * TF;
    if (active && b < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[addr<ILV>(L, c, b + r * nb)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = f + i * TF;
    if (active && b < nb) {
      int g, j;
      if (Ls == 1) {
        g = b;
        j = 0;
      } else {
        g = (int)__umulhi((uint32_t)b, magic);
        j = b - g * Ls;
      }
      if (j != 0) {
        const cx<T>* t = tw + j * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cx<T> w = t[r - 1];
          v[i][r] = (DIR < 0) ? cmul(v[i][r], w) : cmulc(v[i][r], w);
        }
      }
      dft<R, DIR, T>(v[i]);
      const int base = g * Ls * R + j;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[addr<ILV>(L, c, base + r * Ls)] = v[i][r];
    }
  }
  __syncthreads();
}

// Runs all passes of the transform described by d. Every thread of the workgroup must
// call this (passes contain barriers); `active` marks threads that own a transform.
template <int NB, int DIR, bool ILV, typename T>
__device__ void run_fft(cx<T>* buf, const Layout& L, const FftDesc& d, const cx<T>* tw,
                        int c, int f, int TF, bool active) {
  int Ls = 1;
  for (int p = 0; p < d.npass; ++p) {
    const cx<T>* t = tw + d.twoff[p];
    const uint32_t m = d.magic[p];
    switch (d.radix[p]) {
      case 2: stockham_pass<2, NB, DIR, ILV, T>(buf, L, d.P, Ls, m, t, c, f, TF, active); break;
      case 3: stockham_pass<3, NB, DIR, ILV, T>(buf, L, d.P, Ls, m, t, c, f, TF, active); break;
      case 4: stockham_pass<4, NB, DIR, ILV, T>(buf, L, d.P, Ls, m, t, c, f, TF, active); break;
      case 5: stockham_pass<5, NB, DIR, ILV, T>(buf, L, d.P, Ls, m, t, c, f, TF, active); break;
      case 6: stockham_pass<6, NB, DIR, ILV, T>(buf, L, d.P, Ls, m, t, c, f, TF, active); break;
      case 7: stockham_pass<7, NB, DIR, ILV, T>(buf, L, d.P, Ls, m, t, c, f, TF, active); break;
      case 8: stockham_pass<8, NB, DIR, ILV, T>(buf, L, d.P, Ls, m, t, c, f, TF, active); break;
      default: break;  // the host planner never emits other radices
    }
    Ls *= d.radix[p];
  }
}

// Copies the twiddle table of d into LDS (all threads participate; ends with a barrier).
template <typename T>
__device__ __forceinline__ void stage_twiddles(cx<T>* dst, const cx<T>* src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
}

}  // namespace ecc
