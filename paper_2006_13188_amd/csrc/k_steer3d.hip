// Steering in 3D (Sec. 9): spherical-harmonic components of a filter (float64), and the
// per-voxel kernels of the volume path (spectral products, Wigner-D combination and
// modulation).
//
// Conventions: volumes are [z][y][x]; the filter's S^3 array has its centre at (R, R, R)
// and voxel offset q = (x, y, z); polar angle from +z, azimuth atan2(y, x). Spherical
// harmonics are orthonormal with the Condon-Shortley phase, Y_l^m = lam_l^m(cos t) e^{i m p}.
// A rotation R = Rz(alpha) Ry(beta) Rz(gamma) acts on filters by (R F)(x) = F(R^{-1} x), so
// that Y_l^m(R^{-1} x) = sum_m' D^l_{m'm}(R) Y_l^m'(x) with
// D^l_{m'm} = e^{-i m' alpha} d^l_{m'm}(beta) e^{-i m gamma} (Wigner's explicit sum for d).
#include <algorithm>
#include <type_traits>

#include "fft_fixed.hpp"
#include "kcommon.hpp"

namespace ecc {

namespace {

// lam_l^m(t) for one m >= 0 (fully normalised, Condon-Shortley phase): lam_m^m from the
// product formula, then the three-term recurrence in l.
__device__ double sh_lambda(int l, int m, double t) {
  const double s = sqrt(fmax(0.0, 1.0 - t * t));
  double pmm = 0.28209479177387814347;   // 1 / sqrt(4 pi)
  for (int j = 1; j <= m; ++j) pmm = -sqrt((2.0 * j + 1.0) / (2.0 * j)) * s * pmm;
  if (l == m) return pmm;
  double p1 = t * sqrt(2.0 * m + 3.0) * pmm;   // l = m + 1
  double p0 = pmm;
  for (int j = m + 2; j <= l; ++j) {
    const double a = sqrt((4.0 * j * j - 1.0) / ((double)j * j - (double)m * m));
    const double b = sqrt(((double)(j - 1) * (j - 1) - (double)m * m) / (4.0 * (j - 1) * (j - 1) - 1.0));
    const double p2 = a * (t * p1 - b * p0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

__device__ double trilinear64(const float* __restrict__ F, int S, double x, double y, double z) {
  const int R = (S - 1) / 2;
  const double cx_ = x + R, cy = y + R, cz = z + R;
  const double fx0 = floor(cx_), fy0 = floor(cy), fz0 = floor(cz);
  const int ix = (int)fx0, iy = (int)fy0, iz = (int)fz0;
  const double fx = cx_ - fx0, fy = cy - fy0, fz = cz - fz0;
  double acc = 0.0;
  for (int dz = 0; dz < 2; ++dz) {
    const int zz = iz + dz;
    if (zz < 0 || zz >= S) continue;
    const double wz = dz ? fz : 1.0 - fz;
    for (int dy = 0; dy < 2; ++dy) {
      const int yy = iy + dy;
      if (yy < 0 || yy >= S) continue;
      const double wy = dy ? fy : 1.0 - fy;
      for (int dx = 0; dx < 2; ++dx) {
        const int xx = ix + dx;
        if (xx < 0 || xx >= S) continue;
        const double wx = dx ? fx : 1.0 - fx;
        acc += wz * wy * wx * (double)F[((long long)zz * S + yy) * S + xx];
      }
    }
  }
  return acc;
}

// A[ri][i][m] = sum_j F(r_ri w_ij) e^{-i m phi_j}, m = 0..K (negative m: conjugates), on
// the sphere of radius r_ri = sqrt(d2[ri]) at polar node t_i = cos(theta_i) and
// azimuths phi_j = 2 pi j / M.
__global__ void __launch_bounds__(256) k_sh_azimuth(const float* __restrict__ F, int S, int K, int M, int nt,
                                                   const double* __restrict__ gl_t, int nr,
                                                   const int* __restrict__ d2, cx<double>* __restrict__ A) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nr * nt) return;
  const int ri = id / nt, i = id - ri * nt;
  const double r = sqrt((double)d2[ri]);
  const double t = gl_t[i], st = sqrt(fmax(0.0, 1.0 - t * t));
  double are[kMaxSteerK + 1], aim[kMaxSteerK + 1];
#pragma unroll
  for (int m = 0; m <= kMaxSteerK; ++m) are[m] = aim[m] = 0.0;
  for (int j = 0; j < M; ++j) {
    double sp, cp;
    sincospi(2.0 * j / M, &sp, &cp);
    const double v = trilinear64(F, S, r * st * cp, r * st * sp, r * t);
    // e^{-i m phi} by repeated multiplication with e^{-i phi}
    double er = 1.0, ei = 0.0;
#pragma unroll
    for (int m = 0; m <= kMaxSteerK; ++m) {
      if (m <= K) {
        are[m] += v * er;
        aim[m] += v * ei;
      }
      const double nr_ = er * cp + ei * sp, ni = ei * cp - er * sp;
      er = nr_;
      ei = ni;
    }
  }
#pragma unroll
  for (int m = 0; m <= kMaxSteerK; ++m)
    if (m <= K) A[((long long)ri * nt + i) * (K + 1) + m] = mk(are[m], aim[m]);
}

// f[ri][l][m + K] = (2 pi / M) sum_i w_i lam_l^m(t_i) A_m[ri][i] (conj(Y) = lam e^{-i m phi}),
// A_{-m} = conj(A_m) and lam_l^{-m} = (-1)^m lam_l^m.
__global__ void __launch_bounds__(256) k_sh_polar(const cx<double>* __restrict__ A, int nr, int nt, int K, int M,
                                                 const double* __restrict__ gl_t, const double* __restrict__ gl_w,
                                                 cx<double>* __restrict__ f) {
  const int W = 2 * K + 1;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nr * (K + 1) * W) return;
  const int ri = id / ((K + 1) * W), rem = id - ri * (K + 1) * W;
  const int l = rem / W, m = rem % W - K;
  cx<double> out = mk(0.0, 0.0);
  if (m >= -l && m <= l) {
    const int am = m < 0 ? -m : m;
    const double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;
    double sr = 0.0, si = 0.0;
    for (int i = 0; i < nt; ++i) {
      const cx<double> a = A[((long long)ri * nt + i) * (K + 1) + am];
      const double c = gl_w[i] * sh_lambda(l, am, gl_t[i]);
      sr += c * a.re;
      si += c * (m < 0 ? -a.im : a.im);
    }
    const double q = sg * 2.0 * 3.14159265358979323846 / M;
    out = mk(q * sr, q * si);
  }
  f[id] = out;
}

// comps[c][z][y][x] = f_l^m(|q|) Y_l^{m'}(q / |q|) on the ball, the centre F(0) for l = 0.
__global__ void __launch_bounds__(256) k_sh_components(const float* __restrict__ F, int S, int K, int U,
                                                      const int4* __restrict__ hs, const int* __restrict__ rindex,
                                                      const cx<double>* __restrict__ f,
                                                      cx<double>* __restrict__ comps) {
  const long long S3 = (long long)S * S * S;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)U * S3) return;
  const int c = (int)(id / S3);
  const int v = (int)(id - (long long)c * S3);
  const int R = (S - 1) / 2;
  const int iz = v / (S * S), iy = (v / S) % S, ix = v % S;
  const int qx = ix - R, qy = iy - R, qz = iz - R;
  const int d2 = qx * qx + qy * qy + qz * qz;
  const int4 h = hs[c];   // (l, m', m, -)
  cx<double> val = mk(0.0, 0.0);
  if (d2 == 0) {
    if (h.x == 0) val = mk((double)F[v], 0.0);
  } else if (d2 <= R * R) {
    const double r = sqrt((double)d2);
    const double t = qz / r;
    const double ph = atan2((double)qy, (double)qx);
    const double lam = sh_lambda(h.x, h.y, t);
    double sp, cp;
    sincos(h.y * ph, &sp, &cp);
    const cx<double> fc = f[((long long)rindex[d2] * (K + 1) + h.x) * (2 * K + 1) + h.z + K];
    const cx<double> y = mk(lam * cp, lam * sp);
    val = cmul(fc, y);
  }
  comps[id] = val;
}

__global__ void k_real_to_cx(const float* __restrict__ in, cx<float>* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = mk(in[i], 0.0f);
}

// ---- transforms of the volume passes with a compiled schedule (P = R0 R1 R2 with R2 > 1,
// compile-time indexing, the radices and twiddles of fft_fixed.hpp)
//
// These passes are bound by HBM traffic, so the workgroups are small and hold one LDS
// buffer: a transform has NL = P / R2 threads (the last pass is one butterfly per thread,
// whose outputs go straight to memory), which take the earlier passes' butterflies in
// turn; every pass reads all its inputs before a barrier and writes after it.
//
// Columns: kFxB adjacent columns per workgroup, thread (b, c) = (t / kFxB, t % kFxB), so
// every load and store instruction of a wave covers rows of kFxB consecutive complex
// values. in / out: planes (blockIdx.y) of rows with pitch ld; rows j >= nvalid read as
// zero; rows i < nstore are written; mul != NULL multiplies each loaded element by
// mul[j ldIn + v] (the same plane for every input plane).
constexpr int kFxB = 16;

template <class F>
constexpr int fx_rmax() {
  return F::R0 > F::R1 ? (F::R0 > F::R2 ? F::R0 : F::R2) : (F::R1 > F::R2 ? F::R1 : F::R2);
}
template <int N, int T>
constexpr int fx_per_thread() { return (N + T - 1) / T; }

// The three passes on one transform held in LDS at X[pos * ES] (ES = element stride; the
// caller offsets X), driven by thread b < NL. fx_load fetches the first pass's inputs
// from `load(j)` into registers (so that a caller can issue the next transform's loads
// before it runs the current one); fx_passes runs the passes and hands the outputs
// X[b + r NL], r < R2, to `store(r, i = b + r NL, value)`. Threads with act == false take
// part in the barriers only (the caller's other threads).
template <class F>
struct FxIn {
  static constexpr int K0 = fx_per_thread<F::N0, F::N2>();
  cx<float> v[K0][F::R0];
};

template <class F, class Load>
__device__ __forceinline__ void fx_load(FxIn<F>& in, int b, bool act, Load load) {
#pragma unroll
  for (int k = 0; k < FxIn<F>::K0; ++k) {
    const int b0 = b + k * F::N2;
    if (act && b0 < F::N0) {
#pragma unroll
      for (int r = 0; r < F::R0; ++r) in.v[k][r] = load(b0 + r * F::N0);
    }
  }
}

template <class F, int DIR, int ES, class Store>
__device__ __forceinline__ void fx_passes(cx<float>* X, const cx<float>* tw, int b, bool act, FxIn<F>& in,
                                          Store store) {
  static_assert(F::R2 > 1, "three-pass schedules");
  constexpr int NL = F::N2;
  constexpr int K0 = FxIn<F>::K0, K1 = fx_per_thread<F::N1, NL>();
  // pass 0: X[b0 R0 + r] = DFT_R0(in[b0 + r N0])
#pragma unroll
  for (int k = 0; k < K0; ++k) {
    const int b0 = b + k * NL;
    if (act && b0 < F::N0) {
      dft<F::R0, DIR, float>(in.v[k]);
#pragma unroll
      for (int r = 0; r < F::R0; ++r) X[(b0 * F::R0 + r) * ES] = in.v[k][r];
    }
  }
  __syncthreads();
  // pass 1 (Ls = R0)
  cx<float> v1[K1][F::R1];
#pragma unroll
  for (int k = 0; k < K1; ++k) {
    const int b1 = b + k * NL;
    if (act && b1 < F::N1) {
#pragma unroll
      for (int r = 0; r < F::R1; ++r) v1[k][r] = X[(b1 + r * F::N1) * ES];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K1; ++k) {
    const int b1 = b + k * NL;
    if (act && b1 < F::N1) {
      const int j = b1 % F::R0;
      if (j != 0) fixed_twiddle<F::R1, DIR, float>(v1[k], tw + j * (F::R1 - 1));
      dft<F::R1, DIR, float>(v1[k]);
      const int base = (b1 - j) * F::R1 + j;
#pragma unroll
      for (int r = 0; r < F::R1; ++r) X[(base + r * F::R0) * ES] = v1[k][r];
    }
  }
  __syncthreads();
  // pass 2 (Ls = R0 R1, last): one butterfly per thread, natural order out
  if (act) {
    cx<float> v2[F::R2];
#pragma unroll
    for (int r = 0; r < F::R2; ++r) v2[r] = X[(b + r * NL) * ES];
    if (b != 0) fixed_twiddle<F::R2, DIR, float>(v2, tw + F::TW1 + b * (F::R2 - 1));
    dft<F::R2, DIR, float>(v2);
#pragma unroll
    for (int r = 0; r < F::R2; ++r) store(r, b + r * NL, v2[r]);
  }
}

template <class F, int DIR, int ES, class Load, class Store>
__device__ __forceinline__ void fx_transform(cx<float>* X, const cx<float>* tw, int b, bool act, Load load,
                                             Store store) {
  FxIn<F> in;
  fx_load<F>(in, b, act, load);
  fx_passes<F, DIR, ES>(X, tw, b, act, in, store);
}

template <class F, int DIR>
__global__ void __launch_bounds__(F::N2 * kFxB) k_fx_cols(const cx<float>* __restrict__ in, long long planeIn, int ldIn,
                                                        int ncols, int nvalid, cx<float>* __restrict__ out,
                                                        long long planeOut, int ldOut, int nstore,
                                                        const cx<float>* __restrict__ twg,
                                                        const cx<float>* __restrict__ mul) {
  __shared__ cx<float> tw[(F::TW + 1) & ~1];
  __shared__ cx<float> X[F::P * kFxB];
  for (int i = threadIdx.x; i < F::TW; i += blockDim.x) tw[i] = twg[i];
  const int c = threadIdx.x % kFxB, b = threadIdx.x / kFxB;
  const int col = blockIdx.x * kFxB + c;
  const bool cin = col < ncols;
  const cx<float>* src = in + (long long)blockIdx.y * planeIn;
  cx<float>* dst = out + (long long)blockIdx.y * planeOut;
  fx_transform<F, DIR, kFxB>(
      X + c, tw, b, true,
      [&](int j) {
        cx<float> v = mk(0.f, 0.f);
        if (cin && j < nvalid) {
          const long long o = (long long)j * ldIn + col;
          v = src[o];
          if (mul) v = cmul(v, mul[o]);
        }
        return v;
      },
      [&](int, int i, cx<float> v) {
        if (cin && i < nstore) dst[(long long)i * ldOut + col] = v;
      });
}

// Filter spectra kept transformed along x and y only ("partial": the S planes of a
// component's z offsets, offset q_z = j - R in plane j, rows of pitch ld): the column of
// the full spectrum is the transform along z of these planes placed at q_z mod P, so the
// transform's input j is plane (j + R) mod P when that is < S, else zero.
template <class F>
__device__ __forceinline__ cx<float> fx_partial_at(const cx<float>* sp, int ld, int col, bool cin, int S, int R,
                                                   int j) {
  int d = j + R;
  if (d >= F::P) d -= F::P;
  return (cin && d < S) ? sp[(long long)d * ld + col] : mk(0.f, 0.f);
}

// The correlation's inverse z pass with the product formed on chip: per column, the
// filter spectrum column (the transform along z, direction +1, of the component's partial
// planes) times the signal spectrum A, transformed back along z; rows i < nstore of out.
// Component blockIdx.y (partial spectra planeSp apart, outputs planeOut apart); every
// array has row pitch ld.
template <class F>
__global__ void __launch_bounds__(F::N2 * kFxB) k_fx_cols_corr(const cx<float>* __restrict__ sp, long long planeSp,
                                                             int ld, int ncols, int S, int R,
                                                             const cx<float>* __restrict__ A,
                                                             cx<float>* __restrict__ out, long long planeOut,
                                                             int nstore, const cx<float>* __restrict__ twg) {
  __shared__ cx<float> tw[(F::TW + 1) & ~1];
  __shared__ cx<float> X[F::P * kFxB];
  for (int i = threadIdx.x; i < F::TW; i += blockDim.x) tw[i] = twg[i];
  const int c = threadIdx.x % kFxB, b = threadIdx.x / kFxB;
  const int col = blockIdx.x * kFxB + c;
  const bool cin = col < ncols;
  const cx<float>* spc = sp + (long long)blockIdx.y * planeSp;
  cx<float>* dst = out + (long long)blockIdx.y * planeOut;
  // signal spectrum values of this thread's outputs of the first transform (rows b + r NL)
  cx<float> av[F::R2];
#pragma unroll
  for (int r = 0; r < F::R2; ++r) av[r] = cin ? A[(long long)(b + r * F::N2) * ld + col] : mk(0.f, 0.f);
  cx<float> pv[F::R2];
  fx_transform<F, +1, kFxB>(
      X + c, tw, b, true, [&](int j) { return fx_partial_at<F>(spc, ld, col, cin, S, R, j); },
      [&](int r, int, cx<float> v) { pv[r] = cmul(v, av[r]); });
  __syncthreads();   // the last pass's reads of X are done
#pragma unroll
  for (int r = 0; r < F::R2; ++r) X[(b + r * F::N2) * kFxB + c] = pv[r];
  __syncthreads();
  FxIn<F> in;
  fx_load<F>(in, b, true, [&](int j) { return X[j * kFxB + c]; });
  __syncthreads();   // the first pass below rewrites X
  fx_passes<F, +1, kFxB>(X + c, tw, b, true, in, [&](int, int i, cx<float> v) {
    if (cin && i < nstore) dst[(long long)i * ld + col] = v;
  });
}

// Forward column transforms of U planes with the weighted sum of their products with U
// spectra (the convolution's last forward pass and its sum over the components):
// out_g[i][v] = sum_{u in group g} w_u Sp_u[i][v] (DFT of in_u along the rows)[i][v] for
// every i < P, Sp_u and out with row pitch ldOut, in_u rows j >= nvalid zero. Group g =
// blockIdx.y takes components [g per, (g + 1) per) and writes plane g of out (planeOut
// apart); the groups are added by k_sum_planes. Within a group the components are summed
// in order, in registers, so the result does not depend on the launch. PARTIAL: Sp holds
// the partial spectra (S planes of each component, planeSp apart, pitch ldOut), whose
// column is transformed along z (direction -1) on chip before the product.
template <class F, bool PARTIAL = false>
__global__ void __launch_bounds__(F::N2 * kFxB) k_fx_cols_accum(const cx<float>* __restrict__ in, long long planeIn,
                                                              int ldIn, int ncols, int nvalid, int U,
                                                              const cx<float>* __restrict__ Sp, long long planeSp,
                                                              int S, int R, const float* __restrict__ w, int per,
                                                              cx<float>* __restrict__ out, long long planeOut,
                                                              int ldOut, const cx<float>* __restrict__ twg) {
  __shared__ cx<float> tw[(F::TW + 1) & ~1];
  __shared__ cx<float> X[F::P * kFxB];
  for (int i = threadIdx.x; i < F::TW; i += blockDim.x) tw[i] = twg[i];
  const int c = threadIdx.x % kFxB, b = threadIdx.x / kFxB;
  const int col = blockIdx.x * kFxB + c;
  const bool cin = col < ncols;
  cx<float> acc[F::R2];
#pragma unroll
  for (int r = 0; r < F::R2; ++r) acc[r] = mk(0.f, 0.f);
  const int u0 = blockIdx.y * per, u1 = min(U, u0 + per);
  auto loader = [&](int u) {
    const cx<float>* src = in + (long long)u * planeIn;
    return [=](int j) { return cin && j < nvalid ? src[(long long)j * ldIn + col] : mk(0.f, 0.f); };
  };
  // software pipeline: the next component's inputs and this component's spectrum values
  // are requested before this component is transformed
  FxIn<F> cur, nxt;
  if (u0 < u1) fx_load<F>(cur, b, true, loader(u0));
  for (int u = u0; u < u1; ++u) {
    if (u + 1 < u1) fx_load<F>(nxt, b, true, loader(u + 1));
    const cx<float>* sp = Sp + (long long)u * planeSp;
    cx<float> spv[F::R2];
    if constexpr (PARTIAL) {
      fx_transform<F, -1, kFxB>(
          X + c, tw, b, true, [&](int j) { return fx_partial_at<F>(sp, ldOut, col, cin, S, R, j); },
          [&](int r, int, cx<float> v) { spv[r] = v; });
      __syncthreads();   // the signal's transform rewrites X
    } else {
#pragma unroll
      for (int r = 0; r < F::R2; ++r)
        spv[r] = cin ? sp[(long long)(b + r * F::N2) * ldOut + col] : mk(0.f, 0.f);
    }
    const float wu = w[u];
    fx_passes<F, -1, kFxB>(X + c, tw, b, true, cur, [&](int r, int, cx<float> v) {
      const cx<float> p = cmul(v, spv[r]);
      acc[r].re = fmaf(wu, p.re, acc[r].re);
      acc[r].im = fmaf(wu, p.im, acc[r].im);
    });
    __syncthreads();   // the next component rewrites X
    cur = nxt;
  }
  if (cin) {
    cx<float>* dst = out + (long long)blockIdx.y * planeOut;
#pragma unroll
    for (int r = 0; r < F::R2; ++r) dst[(long long)(b + r * F::N2) * ldOut + col] = acc[r];
  }
}

// out[v] = sum_g in[g][v], g = 0..G-1 in order
__global__ void k_sum_planes(const cx<float>* __restrict__ in, long long plane, int G, cx<float>* __restrict__ out,
                             long long n) {
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x) {
    cx<float> a = in[v];
    for (int g = 1; g < G; ++g) a = a + in[(long long)g * plane + v];
    out[v] = a;
  }
}

// Rows: kFxRows rows per workgroup, thread (row, b) = (t / NL, t % NL), each row in its
// own LDS range; consecutive threads read consecutive elements of a row. in / out: planes
// of nrows rows with pitch ld; elements j >= nvalid read as zero, i < nstore written.
constexpr int kFxRows = 8;

template <class F, int DIR>
__global__ void __launch_bounds__(F::N2 * kFxRows) k_fx_rows(const cx<float>* __restrict__ in, long long planeIn,
                                                           int ldIn, int nrows, int nvalid,
                                                           cx<float>* __restrict__ out, long long planeOut,
                                                           int ldOut, int nstore, const cx<float>* __restrict__ twg) {
  __shared__ cx<float> tw[(F::TW + 1) & ~1];
  __shared__ cx<float> X[F::P * kFxRows];
  for (int i = threadIdx.x; i < F::TW; i += blockDim.x) tw[i] = twg[i];
  const int rl = threadIdx.x / F::N2, b = threadIdx.x % F::N2;
  const int row = blockIdx.x * kFxRows + rl;
  const bool act = row < nrows;
  const cx<float>* src = in + (long long)blockIdx.y * planeIn + (long long)(act ? row : 0) * ldIn;
  cx<float>* dst = out + (long long)blockIdx.y * planeOut + (long long)(act ? row : 0) * ldOut;
  fx_transform<F, DIR, 1>(
      X + rl * F::P, tw, b, true,
      [&](int j) { return act && j < nvalid ? src[j] : mk(0.f, 0.f); },
      [&](int, int i, cx<float> v) {
        if (act && i < nstore) dst[i] = v;
      });
}

// the compiled schedules with a volume-pass form (R2 > 1 and NL kFxB <= 1024 threads)
#define ECC_FX3_SIZES(X) X(5, 3, 9)

// A[v] = sum_c w_c X[c][v] Sp[c][v]
__global__ void __launch_bounds__(256) k_spec_accumulate(const cx<float>* __restrict__ X,
                                                        const cx<float>* __restrict__ Sp, const float* __restrict__ w,
                                                        long long V, int U, cx<float>* __restrict__ A) {
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
    float re = 0.f, im = 0.f;
    for (int c = 0; c < U; ++c) {
      const cx<float> p = cmul(X[(long long)c * V + v], Sp[(long long)c * V + v]);
      re = fmaf(w[c], p.re, re);
      im = fmaf(w[c], p.im, im);
    }
    A[v] = mk(re, im);
  }
}

// y[v] = scale Re(in[v])
__global__ void k_real_part(const cx<float>* __restrict__ in, float* __restrict__ y, long long n, float scale) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = in[i].re * scale;
}

// ---- Wigner-D per voxel, with the half-set loops unrolled at compile time
template <int B, int E, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (B < E) {
    fn(std::integral_constant<int, B>{});
    static_for<B + 1, E>(fn);
  }
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cmin(int a, int b) { return a < b ? a : b; }
// terms of Wigner's sum for d^l_{m'm}: k = max(0, m - m') .. min(l + m, l - m')
constexpr int wig_terms(int l, int mp, int m) { return cmin(l + m, l - mp) - cmax(0, m - mp) + 1; }
// half-set order: l = 0..K; m' = 0 with m = 0..l; m' = 1..l with m = -l..l
constexpr int hs_first_m(int mp, int l) { return mp == 0 ? 0 : -l; }
constexpr int hs_index(int l, int mp, int m) {
  int c = 0;
  for (int a = 0; a < l; ++a) c += 2 * a * a + 2 * a + 1;
  for (int b = 0; b < mp; ++b) c += b == 0 ? l + 1 : 2 * l + 1;
  return c + m - hs_first_m(mp, l);
}
constexpr int term_index(int l, int mp, int m) {
  int t = 0;
  for (int a = 0; a <= l; ++a)
    for (int b = 0; b <= a; ++b)
      for (int c = hs_first_m(b, a); c <= a; ++c) {
        if (a == l && b == mp && c == m) return t;
        t += wig_terms(a, b, c);
      }
  return t;
}

// Per-voxel state of the Wigner-D values of the voxel's rotation (float64): powers of
// cos(beta/2) and sin(beta/2), e^{-i m alpha} and e^{-i m gamma} for m = 0..K.
template <int K>
struct WignerVoxel {
  double cpw[2 * K + 1], spw[2 * K + 1];
  double ear[K + 1], eai[K + 1], egr[K + 1], egi[K + 1];
  __device__ __forceinline__ void init(float alpha, float beta, float gamma) {
    double sb, cb, sa, ca, sg, cg;
    sincos(0.5 * (double)beta, &sb, &cb);
    sincos((double)alpha, &sa, &ca);
    sincos((double)gamma, &sg, &cg);
    cpw[0] = spw[0] = 1.0;
#pragma unroll
    for (int j = 1; j <= 2 * K; ++j) {
      cpw[j] = cpw[j - 1] * cb;
      spw[j] = spw[j - 1] * sb;
    }
    ear[0] = egr[0] = 1.0;
    eai[0] = egi[0] = 0.0;
#pragma unroll
    for (int j = 1; j <= K; ++j) {
      ear[j] = ear[j - 1] * ca + eai[j - 1] * sa;
      eai[j] = eai[j - 1] * ca - ear[j - 1] * sa;
      egr[j] = egr[j - 1] * cg + egi[j - 1] * sg;
      egi[j] = egi[j - 1] * cg - egr[j - 1] * sg;
    }
  }
  // D^l_{m'm} = d (pr + i pi): d = d^l_{m'm}(beta) by Wigner's sum (coefficients in the
  // order of term_index), pr + i pi = e^{-i m' alpha} e^{-i m gamma}
  template <int l, int mp, int m>
  __device__ __forceinline__ void entry(const double* __restrict__ coef, double& d, double& pr, double& pi) const {
    constexpr int t0 = term_index(l, mp, m), k0 = cmax(0, m - mp), nk = wig_terms(l, mp, m);
    d = 0.0;
    static_for<0, nk>([&](auto J_) {
      constexpr int k = k0 + decltype(J_)::value;
      d = fma(coef[t0 + decltype(J_)::value], cpw[2 * l + m - mp - 2 * k] * spw[mp - m + 2 * k], d);
    });
    // for m < 0, e^{-i m gamma} = conj(e^{-i |m| gamma})
    constexpr int am = m < 0 ? -m : m;
    const double gr = egr[am], gi = m < 0 ? -egi[am] : egi[am];
    pr = ear[mp] * gr - eai[mp] * gi;
    pi = ear[mp] * gi + eai[mp] * gr;
  }
};

// Calls fn(integral_constant<c>, integral_constant<l>, <m'>, <m>) for every half-set
// component c of band limit K, in order.
template <int K, class Fn>
__device__ __forceinline__ void for_half_set(Fn&& fn) {
  static_for<0, K + 1>([&](auto L_) {
    constexpr int l = decltype(L_)::value;
    static_for<0, l + 1>([&](auto MP_) {
      constexpr int mp = decltype(MP_)::value;
      static_for<hs_first_m(mp, l), l + 1>([&](auto M_) {
        constexpr int m = decltype(M_)::value;
        fn(std::integral_constant<int, hs_index(l, mp, m)>{}, L_, MP_, M_);
      });
    });
  });
}

constexpr int half_set_size(int K) { return (K + 1) * (2 * K * K + 4 * K + 3) / 3; }

// MODE 0 (correlation): y[v] = scale sum_c w_c Re(D_c G_c[v]); MODE 1 (convolution):
// M[c][v] = H[v] D_c. coef: Wigner's coefficients in the order of term_index.
template <int K, int MODE>
__global__ void __launch_bounds__(256) k_wigner_voxels(const float* __restrict__ alpha, const float* __restrict__ beta,
                                                      const float* __restrict__ gamma, long long nvox,
                                                      const double* __restrict__ coef, const float* __restrict__ w,
                                                      const cx<float>* __restrict__ G, const float* __restrict__ H,
                                                      float* __restrict__ y, cx<float>* __restrict__ Mout,
                                                      float scale) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  WignerVoxel<K> wv;
  wv.init(alpha[v], beta[v], gamma[v]);
  const float h = MODE == 1 ? H[v] : 0.f;
  float acc = 0.f;
  for_half_set<K>([&](auto C_, auto L_, auto MP_, auto M_) {
    constexpr int c = decltype(C_)::value;
    double d, pr, pi;
    wv.template entry<decltype(L_)::value, decltype(MP_)::value, decltype(M_)::value>(coef, d, pr, pi);
    if constexpr (MODE == 0) {
      const cx<float> g = G[(long long)c * nvox + v];
      // Re(D G) = d (pr g.re - pi g.im)
      acc = fmaf(w[c] * (float)d, (float)pr * g.re - (float)pi * g.im, acc);
    } else {
      Mout[(long long)c * nvox + v] = mk((float)(d * pr) * h, (float)(d * pi) * h);
    }
  });
  if constexpr (MODE == 0) y[v] = acc * scale;
}

// The correlation's last inverse pass (along x) fused with the Wigner-D combination, for a
// compiled transform length: one workgroup per output row (z, y). Its components' rows are
// transformed kFxCh at a time (kFxCh groups of NL threads, one row each) into LDS, then
// thread x (one output voxel) adds w_c Re(D_c(x) G_c(x)) for those components; the
// component loop is unrolled, so every D entry has constant indices. in: component planes
// (planeIn apart) of nrows rows with pitch ldIn, nvalid valid elements per row; y: rows of
// nx voxels; alpha, beta, gamma: the same layout as y.
constexpr int kFxCh = 8;

template <class F, int K>
__global__ void __launch_bounds__(192) k_fx_rows_wigner(const cx<float>* __restrict__ in, long long planeIn, int ldIn,
                                                       int nvalid, int nx, const float* __restrict__ alpha,
                                                       const float* __restrict__ beta, const float* __restrict__ gamma,
                                                       const double* __restrict__ coef, const float* __restrict__ w,
                                                       float* __restrict__ y, float scale,
                                                       const cx<float>* __restrict__ twg) {
  constexpr int NL = F::N2, U = half_set_size(K), NCH = (U + kFxCh - 1) / kFxCh;
  static_assert(kFxCh * NL <= 192, "one row transform per thread group");
  __shared__ cx<float> tw[(F::TW + 1) & ~1];
  __shared__ cx<float> X[kFxCh * F::P];
  __shared__ cx<float> Gs[kFxCh * F::P];
  for (int i = threadIdx.x; i < F::TW; i += blockDim.x) tw[i] = twg[i];
  const int t = threadIdx.x;
  const int kk = t / NL, b = t - kk * NL;   // transform role: component slot kk of a chunk
  const long long row = blockIdx.x;
  const bool vox = t < nx;                  // voxel role: x = t
  const long long p = row * nx + t;
  WignerVoxel<K> wv;
  if (vox) wv.init(alpha[p], beta[p], gamma[p]);
  float acc = 0.f;
  auto active = [&](int c0) { return kk < kFxCh && c0 + kk < U; };
  auto loader = [&](int c0) {
    const cx<float>* src = in + (long long)(active(c0) ? c0 + kk : 0) * planeIn + row * ldIn;
    return [=](int j) { return j < nvalid ? src[j] : mk(0.f, 0.f); };
  };
  // software pipeline: the next chunk's rows are requested before this chunk is transformed
  FxIn<F> cur, nxt;
  fx_load<F>(cur, b, active(0), loader(0));
  static_for<0, NCH>([&](auto CH_) {
    constexpr int c0 = decltype(CH_)::value * kFxCh;
    if constexpr (c0 + kFxCh < U) fx_load<F>(nxt, b, active(c0 + kFxCh), loader(c0 + kFxCh));
    fx_passes<F, +1, 1>(X + (kk < kFxCh ? kk : 0) * F::P, tw, b, active(c0), cur,
                        [&](int, int i, cx<float> v) { Gs[kk * F::P + i] = v; });
    __syncthreads();   // the chunk's rows are in Gs
    if (vox) {
      for_half_set<K>([&](auto C_, auto L_, auto MP_, auto M_) {
        constexpr int cc = decltype(C_)::value;
        if constexpr (cc >= c0 && cc < c0 + kFxCh) {
          double d, pr, pi;
          wv.template entry<decltype(L_)::value, decltype(MP_)::value, decltype(M_)::value>(coef, d, pr, pi);
          const cx<float> g = Gs[(cc - c0) * F::P + t];
          acc = fmaf(w[cc] * (float)d, (float)pr * g.re - (float)pi * g.im, acc);
        }
      });
    }
    __syncthreads();   // Gs and X are rewritten by the next chunk
    cur = nxt;
  });
  if (vox) y[p] = acc * scale;
}

}  // namespace

hipError_t launch_sh_azimuth(hipStream_t s, const float* F, int S, int K, int M, int nt, const double* gl_t, int nr,
                             const int* d2, cx<double>* A) {
  if (K < 0 || K > kMaxSteerK) return hipErrorInvalidValue;
  const int n = nr * nt;
  hipLaunchKernelGGL(k_sh_azimuth, dim3((n + 255) / 256), dim3(256), 0, s, F, S, K, M, nt, gl_t, nr, d2, A);
  return last();
}

hipError_t launch_sh_polar(hipStream_t s, const cx<double>* A, int nr, int nt, int K, int M, const double* gl_t,
                           const double* gl_w, cx<double>* f) {
  const int n = nr * (K + 1) * (2 * K + 1);
  hipLaunchKernelGGL(k_sh_polar, dim3((n + 255) / 256), dim3(256), 0, s, A, nr, nt, K, M, gl_t, gl_w, f);
  return last();
}

hipError_t launch_sh_components(hipStream_t s, const float* F, int S, int K, int U, const int4* hs,
                                const int* rindex, const cx<double>* f, cx<double>* comps) {
  const long long n = (long long)U * S * S * S;
  hipLaunchKernelGGL(k_sh_components, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, F, S, K, U, hs, rindex,
                     f, comps);
  return last();
}

static unsigned grid_for(long long n) {
  const long long b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

hipError_t launch_real_to_cx(hipStream_t s, const float* in, cx<float>* out, long long n) {
  hipLaunchKernelGGL(k_real_to_cx, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return last();
}

bool fx3_supported(int P) {
#define ECC_FXS(a, b_, c_) \
  if (P == (a) * (b_) * (c_)) return true;
  ECC_FX3_SIZES(ECC_FXS)
#undef ECC_FXS
  return false;
}

hipError_t launch_fx_cols(hipStream_t s, int P, int dir, int nplanes, const cx<float>* in, long long planeIn,
                          int ldIn, int ncols, int nvalid, cx<float>* out, long long planeOut, int ldOut,
                          int nstore, const cx<float>* tw, const cx<float>* mul) {
#define ECC_FXC(a, b_, c_)                                                                         \
  if (P == (a) * (b_) * (c_)) {                                                                    \
    using F = Fixed3<a, b_, c_>;                                                                   \
    if (nvalid > P || nstore > P) return hipErrorInvalidValue;                                     \
    const dim3 g((ncols + kFxB - 1) / kFxB, nplanes), blk(F::N2 * kFxB);                           \
    if (dir < 0)                                                                                   \
      hipLaunchKernelGGL((k_fx_cols<F, -1>), g, blk, 0, s, in, planeIn, ldIn, ncols, nvalid, out,  \
                         planeOut, ldOut, nstore, tw, mul);                                        \
    else                                                                                           \
      hipLaunchKernelGGL((k_fx_cols<F, +1>), g, blk, 0, s, in, planeIn, ldIn, ncols, nvalid, out,  \
                         planeOut, ldOut, nstore, tw, mul);                                        \
    return last();                                                                                 \
  }
  ECC_FX3_SIZES(ECC_FXC)
#undef ECC_FXC
  return hipErrorInvalidValue;
}

hipError_t launch_fx_rows(hipStream_t s, int P, int dir, int nplanes, const cx<float>* in, long long planeIn,
                          int ldIn, int nrows, int nvalid, cx<float>* out, long long planeOut, int ldOut,
                          int nstore, const cx<float>* tw) {
#define ECC_FXR(a, b_, c_)                                                                          \
  if (P == (a) * (b_) * (c_)) {                                                                     \
    using F = Fixed3<a, b_, c_>;                                                                    \
    if (nvalid > P || nstore > P) return hipErrorInvalidValue;                                      \
    const dim3 g((nrows + kFxRows - 1) / kFxRows, nplanes), blk(F::N2 * kFxRows);                    \
    if (dir < 0)                                                                                    \
      hipLaunchKernelGGL((k_fx_rows<F, -1>), g, blk, 0, s, in, planeIn, ldIn, nrows, nvalid, out,   \
                         planeOut, ldOut, nstore, tw);                                              \
    else                                                                                            \
      hipLaunchKernelGGL((k_fx_rows<F, +1>), g, blk, 0, s, in, planeIn, ldIn, nrows, nvalid, out,   \
                         planeOut, ldOut, nstore, tw);                                              \
    return last();                                                                                  \
  }
  ECC_FX3_SIZES(ECC_FXR)
#undef ECC_FXR
  return hipErrorInvalidValue;
}

hipError_t launch_fx_cols_corr(hipStream_t s, int P, int nplanes, const cx<float>* sp, long long planeSp, int ld,
                               int ncols, int S, int R, const cx<float>* A, cx<float>* out, long long planeOut,
                               int nstore, const cx<float>* tw) {
#define ECC_FXK(a, b_, c_)                                                                            \
  if (P == (a) * (b_) * (c_)) {                                                                       \
    using F = Fixed3<a, b_, c_>;                                                                      \
    if (S != 2 * R + 1 || S > P || nstore > P || nplanes < 1 || nplanes > 65535) return hipErrorInvalidValue; \
    hipLaunchKernelGGL((k_fx_cols_corr<F>), dim3((ncols + kFxB - 1) / kFxB, nplanes), dim3(F::N2 * kFxB), 0, \
                       s, sp, planeSp, ld, ncols, S, R, A, out, planeOut, nstore, tw);                \
    return last();                                                                                    \
  }
  ECC_FX3_SIZES(ECC_FXK)
#undef ECC_FXK
  return hipErrorInvalidValue;
}

hipError_t launch_fx_cols_accum(hipStream_t s, int P, int nplanes, const cx<float>* in, long long planeIn, int ldIn,
                                int ncols, int nvalid, const cx<float>* Sp, long long planeSp, int S, int R,
                                const float* w, int groups, cx<float>* part, long long planePart, cx<float>* out,
                                int ldOut, const cx<float>* tw) {
#define ECC_FXA(a, b_, c_)                                                                          \
  if (P == (a) * (b_) * (c_)) {                                                                     \
    using F = Fixed3<a, b_, c_>;                                                                    \
    if (nvalid > P || nplanes < 1 || groups < 1 || (S > 0 && (S != 2 * R + 1 || S > P)))            \
      return hipErrorInvalidValue;                                                                  \
    const int per = (nplanes + groups - 1) / groups, G = (nplanes + per - 1) / per;                 \
    cx<float>* dst = G > 1 ? part : out;                                                            \
    const dim3 g((ncols + kFxB - 1) / kFxB, G), blk(F::N2 * kFxB);                                  \
    if (S > 0)                                                                                      \
      hipLaunchKernelGGL((k_fx_cols_accum<F, true>), g, blk, 0, s, in, planeIn, ldIn, ncols, nvalid, nplanes, \
                         Sp, planeSp, S, R, w, per, dst, planePart, ldOut, tw);                     \
    else                                                                                            \
      hipLaunchKernelGGL((k_fx_cols_accum<F>), g, blk, 0, s, in, planeIn, ldIn, ncols, nvalid, nplanes, Sp, \
                         planeSp, 0, 0, w, per, dst, planePart, ldOut, tw);                         \
    if (G > 1) {                                                                                    \
      hipError_t e = last();                                                                        \
      if (e != hipSuccess) return e;                                                                \
      const long long n = (long long)P * ldOut;                                                     \
      hipLaunchKernelGGL(k_sum_planes, dim3(grid_for(n)), dim3(256), 0, s, part, planePart, G, out, n); \
    }                                                                                               \
    return last();                                                                                  \
  }
  ECC_FX3_SIZES(ECC_FXA)
#undef ECC_FXA
  return hipErrorInvalidValue;
}

bool fx_rows_wigner_supported(int P, int K, int nx) {
  return fx3_supported(P) && K >= 0 && K <= kFusedWignerK && nx >= 1 && nx <= 192;
}

hipError_t launch_fx_rows_wigner(hipStream_t s, int P, int K, const cx<float>* in, long long planeIn, int ldIn,
                                 int nrows, int nvalid, int nx, const float* alpha, const float* beta,
                                 const float* gamma, const double* coef, const float* w, float* y, float scale,
                                 const cx<float>* tw) {
  if (!fx_rows_wigner_supported(P, K, nx) || nvalid > P || nrows < 1) return hipErrorInvalidValue;
  const unsigned nthr = (unsigned)((std::max(kFxCh * 15, nx) + 63) / 64 * 64);
#define ECC_FXW(a, b_, c_)                                                                               \
  if (P == (a) * (b_) * (c_)) {                                                                          \
    using F = Fixed3<a, b_, c_>;                                                                         \
    static_assert(F::N2 == 15, "thread count above assumes 15 threads per row transform");              \
    switch (K) {                                                                                         \
      case 0: hipLaunchKernelGGL((k_fx_rows_wigner<F, 0>), dim3(nrows), dim3(nthr), 0, s, in, planeIn, ldIn, nvalid, nx, alpha, beta, gamma, coef, w, y, scale, tw); break; \
      case 1: hipLaunchKernelGGL((k_fx_rows_wigner<F, 1>), dim3(nrows), dim3(nthr), 0, s, in, planeIn, ldIn, nvalid, nx, alpha, beta, gamma, coef, w, y, scale, tw); break; \
      case 2: hipLaunchKernelGGL((k_fx_rows_wigner<F, 2>), dim3(nrows), dim3(nthr), 0, s, in, planeIn, ldIn, nvalid, nx, alpha, beta, gamma, coef, w, y, scale, tw); break; \
      case 3: hipLaunchKernelGGL((k_fx_rows_wigner<F, 3>), dim3(nrows), dim3(nthr), 0, s, in, planeIn, ldIn, nvalid, nx, alpha, beta, gamma, coef, w, y, scale, tw); break; \
      case 4: hipLaunchKernelGGL((k_fx_rows_wigner<F, 4>), dim3(nrows), dim3(nthr), 0, s, in, planeIn, ldIn, nvalid, nx, alpha, beta, gamma, coef, w, y, scale, tw); break; \
      default: return hipErrorInvalidValue;                                                              \
    }                                                                                                    \
    return last();                                                                                       \
  }
  ECC_FX3_SIZES(ECC_FXW)
#undef ECC_FXW
  return hipErrorInvalidValue;
}

hipError_t prepare_fx_kernels() { return hipSuccess; }   // static LDS only

hipError_t launch_spec_accumulate(hipStream_t s, const cx<float>* X, const cx<float>* Sp, const float* w, long long V,
                                  int U, cx<float>* A) {
  hipLaunchKernelGGL(k_spec_accumulate, dim3(grid_for(V)), dim3(256), 0, s, X, Sp, w, V, U, A);
  return last();
}

hipError_t launch_real_part(hipStream_t s, const cx<float>* in, float* y, long long n, float scale) {
  hipLaunchKernelGGL(k_real_part, dim3(grid_for(n)), dim3(256), 0, s, in, y, n, scale);
  return last();
}

hipError_t launch_wigner_voxels(hipStream_t s, int K, int mode, const float* alpha, const float* beta,
                                const float* gamma, long long nvox, const double* coef, const float* w,
                                const cx<float>* G, const float* H, float* y, cx<float>* M, float scale) {
  const dim3 g((unsigned)((nvox + 255) / 256)), b(256);
#define ECC_WV(KK)                                                                                        \
  case KK:                                                                                                \
    if (mode == 0)                                                                                        \
      hipLaunchKernelGGL((k_wigner_voxels<KK, 0>), g, b, 0, s, alpha, beta, gamma, nvox, coef, w, G, H, y, M, \
                         scale);                                                                          \
    else                                                                                                  \
      hipLaunchKernelGGL((k_wigner_voxels<KK, 1>), g, b, 0, s, alpha, beta, gamma, nvox, coef, w, G, H, y, M, \
                         scale);                                                                          \
    break;
  switch (K) {
    ECC_WV(0) ECC_WV(1) ECC_WV(2) ECC_WV(3) ECC_WV(4) ECC_WV(5) ECC_WV(6) ECC_WV(7) ECC_WV(8)
    default:
      return hipErrorInvalidValue;
  }
#undef ECC_WV
  return last();
}

}  // namespace ecc
