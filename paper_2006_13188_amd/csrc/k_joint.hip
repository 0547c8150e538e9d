// Joint rotation and scale fields (the Conclusion's product-group extension): the plan's
// components F_{k,l}(x) = c_{k,l} e^{i k phi(x)} e^{i omega_l (ln|x| - u_lo)} from log-polar
// samples of the filter (float64), and the modulated row transforms of the two-pass
// extended convolution with the phase e^{-i (k theta(q) + omega_l ln s(q))}.
#include "kcommon.hpp"

namespace ecc {

namespace {

__device__ double bilinear_joint(const float* F, int S, double dx, double dy) {
  const int R = (S - 1) / 2;
  const double col = dx + R, row = dy + R;
  const int c0 = (int)floor(col), r0 = (int)floor(row);
  const double fc = col - c0, fr = row - r0;
  double acc = 0.0;
  for (int a = 0; a < 2; ++a) {
    const int rr = r0 + a;
    const double wr = a ? fr : 1.0 - fr;
    if (rr < 0 || rr >= S) continue;
    for (int b = 0; b < 2; ++b) {
      const int cc = c0 + b;
      const double wc = b ? fc : 1.0 - fc;
      if (cc < 0 || cc >= S) continue;
      acc += wr * wc * (double)F[rr * S + cc];
    }
  }
  return acc;
}

// One block per log radius: j < n at u_lo + j L / n, j = n at u_hi, j = n + 1 at u_lo.
// f[j][k + K] = (1/M) sum_m F(e^u cos phi_m, e^u sin phi_m) e^{-i k phi_m}, zero beyond R.
__global__ void __launch_bounds__(256) k_joint_samples(const float* __restrict__ F, int S, int K, int M, int n,
                                                      double u_lo, double u_hi, double L,
                                                      cx<double>* __restrict__ f) {
  extern __shared__ double smem_j[];
  double* v = smem_j;
  double* ct = v + M;
  double* st = ct + M;
  const int j = blockIdx.x;
  const int R = (S - 1) / 2;
  const double u = j < n ? u_lo + (double)j * L / (double)n : (j == n ? u_hi : u_lo);
  const double r = exp(u);
  const bool inside = r <= (double)R + 1e-9;
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)M, &sn, &cs);
    ct[m] = cs;
    st[m] = sn;
    v[m] = inside ? bilinear_joint(F, S, r * cs, r * sn) : 0.0;
  }
  __syncthreads();
  for (int kk = threadIdx.x; kk <= 2 * K; kk += blockDim.x) {
    const int k = kk - K;
    const int step = ((k % M) + M) % M;
    double re = 0.0, im = 0.0;
    int t = 0;
    for (int m = 0; m < M; ++m) {
      re += v[m] * ct[t];
      im -= v[m] * st[t];
      t += step;
      if (t >= M) t -= M;
    }
    cx<double> o;
    o.re = re / (double)M;
    o.im = im / (double)M;
    f[(long long)j * (2 * K + 1) + kk] = o;
  }
}

// c[k + K][l + h] = (1/n) sum_j h_k(u_j) e^{-2 pi i j l / n}, h_k(u_j) = f_k(e^{u_j}) on
// [u_lo, u_hi] and a raised cosine from f_k(e^{u_hi}) back to f_k(e^{u_lo}) beyond.
__global__ void __launch_bounds__(256) k_joint_coeffs(const cx<double>* __restrict__ f, int K, int n, double u_lo,
                                                     double u_hi, double L, cx<double>* __restrict__ c) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int nk = 2 * K + 1;
  if (idx >= nk * n) return;
  const int kk = idx / n, a = idx - kk * n, h = (n - 1) / 2, l = a - h;
  const cx<double> fhi = f[(long long)n * nk + kk], flo = f[(long long)(n + 1) * nk + kk];
  double re = 0.0, im = 0.0;
  for (int j = 0; j < n; ++j) {
    const double u = u_lo + (double)j * L / (double)n;
    cx<double> hv;
    if (u <= u_hi + 1e-12) {
      hv = f[(long long)j * nk + kk];
    } else {
      const double t = (u - u_hi) / (u_lo + L - u_hi);
      const double b = 0.5 * (1.0 - cospi(t));
      hv.re = fhi.re + (flo.re - fhi.re) * b;
      hv.im = fhi.im + (flo.im - fhi.im) * b;
    }
    double sn, cs;
    sincospi(-2.0 * (double)(((long long)j * l) % n) / (double)n, &sn, &cs);
    re += hv.re * cs - hv.im * sn;
    im += hv.re * sn + hv.im * cs;
  }
  c[idx].re = re / (double)n;
  c[idx].im = im / (double)n;
}

// component c = (k, l) of the half set: k = 0 with l = 0..h, then k = 1..K with l = -h..h
__device__ __forceinline__ void joint_kl(int c, int n, int* k, int* l) {
  const int h = (n - 1) / 2;
  if (c <= h) {
    *k = 0;
    *l = c;
  } else {
    const int d = c - (h + 1);
    *k = 1 + d / n;
    *l = d % n - h;
  }
}

__global__ void __launch_bounds__(256) k_joint_synth(const float* __restrict__ F, int S, int K, int n, int U,
                                                    double u_lo, double om1, const cx<double>* __restrict__ c,
                                                    cx<double>* __restrict__ comps) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int np = S * S;
  if (idx >= U * np) return;
  const int ci = idx / np, p = idx - ci * np;
  int k, l;
  joint_kl(ci, n, &k, &l);
  const int R = (S - 1) / 2, h = (n - 1) / 2;
  const int dy = p / S - R, dx = p % S - R;
  const int r2 = dx * dx + dy * dy;
  cx<double> o;
  o.re = 0.0;
  o.im = 0.0;
  if (r2 == 0) {
    if (k == 0 && l == 0) o.re = (double)F[p];
  } else if (r2 <= R * R) {
    const cx<double> cv = c[(long long)(k + K) * n + (l + h)];
    const double ang = (double)k * atan2((double)dy, (double)dx) + om1 * (double)l * (0.5 * log((double)r2) - u_lo);
    double sn, cs;
    sincos(ang, &sn, &cs);
    o.re = cv.re * cs - cv.im * sn;
    o.im = cv.re * sn + cv.im * cs;
  }
  comps[idx] = o;
}

// Modulated row transforms of the two-pass convolution for joint fields:
// B_{c,s} = FFT_x(sig_s e^{-i (k_c theta + omega_{l_c} ln s)}), sig_0 = H wn, sig_1 = wn
// (wn = 1 / s^2 with sig_norm, else 1). The phase is kept as two float64 recurrences along
// the component order: e^{-i k theta} (once per k) and e^{-i omega_l ln s} (once per l,
// restarting at l = -h for every k >= 1).
template <int NB, int EPX>
__global__ void __launch_bounds__(256) k_conv_rows_fwd_joint(
    const float* __restrict__ H, long long planeH, int ldH, JointField jf, int sig_norm, int nsig,
    cx<float>* __restrict__ Bk, long long planeBk, long long planeBsig, long long planeBimg, int ldB,
    int ny, int nx, int U, int n, FftDesc d, const cx<float>* __restrict__ tw, int B, int TF) {
  extern __shared__ cx<float> smem_f[];
  cx<float>* twl = smem_f;
  cx<float>* buf = smem_f + lds_tw_pad(d.twsize);
  stage_twiddles(twl, tw, d.twsize);
  const int Px = d.P;
  const int c = threadIdx.x / TF, f = threadIdx.x - c * TF;
  const int row = blockIdx.x * B + c;
  const bool active = (c < B) && (row < ny);
  const int img = blockIdx.y;
  const int h = (n - 1) / 2;
  Layout Lo{B, 0, Px};
  Phase et[EPX], es[EPX], zs0[EPX], zk[EPX], zl[EPX];
  double sg[2][EPX];
#pragma unroll
  for (int j = 0; j < EPX; ++j) {
    const int x = f + j * TF;
    Phase one;
    one.re = 1.0;
    one.im = 0.0;
    et[j] = es[j] = zs0[j] = zk[j] = zl[j] = one;
    sg[0][j] = 0.0;
    sg[1][j] = 0.0;
    if (active && x < nx) {
      const float th = jf.theta[(long long)img * jf.plane_t + (long long)row * jf.ld_t + x];
      const float sv = jf.scale[(long long)img * jf.plane_s + (long long)row * jf.ld_s + x];
      const double ls = log((double)sv);
      double sn, cs;
      sincos((double)th, &sn, &cs);
      et[j].re = cs;
      et[j].im = -sn;   // e^{-i theta}
      sincos(jf.om1 * ls, &sn, &cs);
      es[j].re = cs;
      es[j].im = -sn;   // e^{-i omega_1 ln s}
      sincos(jf.om1 * (double)h * ls, &sn, &cs);
      zs0[j].re = cs;
      zs0[j].im = sn;   // e^{+i omega_h ln s}: the phase of l = -h
      const double h0 = (double)H[(long long)img * planeH + (long long)row * ldH + x];
      const double wn = sig_norm ? 1.0 / ((double)sv * (double)sv) : 1.0;
      sg[0][j] = h0 * wn;
      sg[1][j] = wn;
    }
  }
  for (int ci = 0; ci < U; ++ci) {
    int k, l;
    joint_kl(ci, n, &k, &l);
    if (ci > 0) {
      if (l == (k == 0 ? 0 : -h)) {   // a new angular frequency
#pragma unroll
        for (int j = 0; j < EPX; ++j) {
          zk[j] = pmul(zk[j], et[j]);
          zl[j] = zs0[j];
        }
      } else {
#pragma unroll
        for (int j = 0; j < EPX; ++j) zl[j] = pmul(zl[j], es[j]);
      }
    }
    for (int s = 0; s < nsig; ++s) {
      if (active) {
        for (int pos = nx + f; pos < Px; pos += TF) buf[c * Px + pos] = mk(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < EPX; ++j) {
          const int x = f + j * TF;
          if (x < nx) {
            const Phase z = pmul(zk[j], zl[j]);
            buf[c * Px + x] = mk((float)(sg[s][j] * z.re), (float)(sg[s][j] * z.im));
          }
        }
      }
      __syncthreads();
      run_fft<NB, -1, false, float>(buf, Lo, d, twl, c, f, TF, active);
      if (active) {
        cx<float>* dst = Bk + (long long)img * planeBimg + (long long)s * planeBsig + (long long)ci * planeBk +
                         (long long)row * ldB;
        for (int pos = f; pos < Px; pos += TF) dst[pos] = buf[c * Px + pos];
      }
      __syncthreads();   // the next signal overwrites positions other threads just stored
    }
  }
}

}  // namespace

hipError_t launch_joint_components(hipStream_t s, const float* F, int S, int K, int M, int n, double u_lo,
                                   double u_hi, double L, cx<double>* f_tmp, cx<double>* c_tmp, cx<double>* comps) {
  const int nk = 2 * K + 1, U = (K + 1) * n - (n - 1) / 2;
  hipLaunchKernelGGL(k_joint_samples, dim3(n + 2), dim3(256), 3 * (size_t)M * sizeof(double), s, F, S, K, M, n,
                     u_lo, u_hi, L, f_tmp);
  hipError_t e = last();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_joint_coeffs, dim3((unsigned)((nk * n + 255) / 256)), dim3(256), 0, s, f_tmp, K, n, u_lo,
                     u_hi, L, c_tmp);
  if ((e = last()) != hipSuccess) return e;
  const long long tot = (long long)U * S * S;
  hipLaunchKernelGGL(k_joint_synth, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, F, S, K, n, U, u_lo,
                     2.0 * 3.14159265358979323846 / L, c_tmp, comps);
  return last();
}

hipError_t launch_conv_rows_fwd_joint(hipStream_t s, const RowCfg& c, int batch, const float* H, long long planeH,
                                      int ldH, const JointField& jf, int sig_norm, int nsig, cx<float>* Bk,
                                      long long planeBk, long long planeBsig, long long planeBimg, int ldB, int ny,
                                      int nx, int U, int n, const FftDesc& d, const cx<float>* tw) {
  if (c.B * c.TF > 256) return hipErrorInvalidValue;   // the kernel's launch bound
  dim3 grid((ny + c.B - 1) / c.B, batch), block(c.B * c.TF);
  const size_t lds = lds_rows(c, d, sizeof(cx<float>));
  ECC_NB_SWITCH(c.NB, ECC_EPX_SWITCH(c.EPX, hipLaunchKernelGGL((k_conv_rows_fwd_joint<NB, EPX>), grid, block, lds,
                                                               s, H, planeH, ldH, jf, sig_norm, nsig, Bk, planeBk,
                                                               planeBsig, planeBimg, ldB, ny, nx, U, n, d, tw, c.B,
                                                               c.TF)));
  return last();
}

}  // namespace ecc
