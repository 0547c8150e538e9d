// C-ABI of steering in 3D (Sec. 9): volume plans (spherical-harmonic components of a
// filter, their spectra) and the extended correlation / convolution of volumes with a
// per-voxel rotation field.
#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "api_common.hpp"

using namespace ecc;

struct ecc_volume_plan_s {
  ecc_context ctx = nullptr;
  int device = 0;
  int S = 0, R = 0, K = 0, U = 0, M = 0;
  std::vector<int4> hs;          // (l, m', m, 0) per component, half-set order
  std::vector<float> weights;    // 1 for (l, 0, 0), else 2
  DevBuf d_w;                    // weights on the device
  DevBuf coef;                   // Wigner's coefficients (float64), term order
  DevBuf comps64;                // U x S^3 complex128
  DevBuf comps32;                // U x S^3 complex64
  std::mutex mu;
  std::map<std::tuple<int, int, int, int>, std::unique_ptr<DevBuf>> spectra;   // (op, Pz, Py, Px)
};

namespace ecc {
void destroy_volume_plans(ecc_context ctx) {
  for (ecc_volume_plan p : ctx->vplans) delete p;
  ctx->vplans.clear();
}
}  // namespace ecc

namespace {

inline hipStream_t S_(void* s) { return static_cast<hipStream_t>(s); }

constexpr int kMaxSteerS = 63;
constexpr int kMaxPlanes = 65535;   // grid.y limit of the generic transforms
// column passes: 2^kColLgB adjacent columns per workgroup of kColThreads threads
constexpr int kColLgB = 4, kColThreads = 512;

// Gauss-Legendre nodes and weights on [-1, 1] (Newton's iteration on P_n, long double).
void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& w) {
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    long double x = cosl(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // P_n = p1, P_{n-1} = p0; P_n' = n (x P_n - P_{n-1}) / (x^2 - 1)
      dp = n * (x * p1 - p0) / (x * x - 1);
      const long double dx = p1 / dp;
      x -= dx;
      if (fabsl(dx) < 1e-19L) break;
    }
    {
      long double p0 = 1, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1);
    }
    const long double wi = 2.0L / ((1 - x * x) * dp * dp);
    t[i] = (double)x;
    t[n - 1 - i] = (double)-x;
    w[i] = w[n - 1 - i] = (double)wi;
  }
  if (n % 2) t[n / 2] = 0.0;
}

long double lfact(int n) {
  long double r = 1;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

int azimuths(int K, int R) {
  const int need = std::max(8 * (2 * K + 1), 4 * (int)std::ceil(2.0 * 3.14159265358979323846 * R));
  int M = 1;
  while (M < need) M *= 2;
  return M;
}

ecc_status check_row(const RowCfg& c, const Transform& t, size_t elem) {
  if (c.NB < 0 || c.EPX < 0 || lds_rows(c, t.desc, elem) > kMaxLds)
    return fail(ECC_ERR_UNSUPPORTED, "transform too long for the row kernel");
  return ECC_OK;
}
ecc_status check_col(const ColCfg& c, const Transform& t, size_t elem) {
  if (c.NB < 0 || lds_cols(c, t.desc, elem) > kMaxLds)
    return fail(ECC_ERR_UNSUPPORTED, "transform too long for the column kernel");
  return ECC_OK;
}

// Transforms along the three axes of a batch of volumes, planes split to respect the
// grid limit. Rows (x): every plane holds `nrows` rows.
// (float32 passes of a length with a compiled schedule take the fixed-schedule kernels)
template <typename T>
ecc_status rows_pass(hipStream_t st, const Transform& tr, int nplanes, int dir, const cx<T>* in, long long pIn,
                     int ldIn, int nrows, int nvalid, int shift, cx<T>* out, long long pOut, int ldOut, int nstore) {
  if constexpr (sizeof(T) == 4) {
    if (shift == 0 && tr.fR0 && fx3_supported(tr.desc.P)) {
      for (int p0 = 0; p0 < nplanes; p0 += kMaxPlanes) {
        const int np = std::min(kMaxPlanes, nplanes - p0);
        ECC_HIP(launch_fx_rows(st, tr.desc.P, dir, np, in + p0 * pIn, pIn, ldIn, nrows, nvalid, out + p0 * pOut,
                               pOut, ldOut, nstore, tr.fx()));
      }
      return ECC_OK;
    }
  }
  const RowCfg rc = row_config(tr, tr.desc.P, sizeof(cx<T>));
  ECC_TRY(check_row(rc, tr, sizeof(cx<T>)));
  for (int p0 = 0; p0 < nplanes; p0 += kMaxPlanes) {
    const int np = std::min(kMaxPlanes, nplanes - p0);
    ECC_HIP((launch_fft_rows<T>(st, rc, np, dir, in + p0 * pIn, pIn, ldIn, nrows, nvalid, shift, out + p0 * pOut,
                                pOut, ldOut, nstore, 0, tr.desc, sizeof(T) == 8 ? (const cx<T>*)tr.d() : (const cx<T>*)tr.f())));
  }
  return ECC_OK;
}
// Columns: transform along the rows of planes of `ncols` columns with row pitch ld.
template <typename T>
ecc_status cols_pass(hipStream_t st, const Transform& tr, int nplanes, int dir, const cx<T>* in, long long pIn,
                     int ldIn, int ncols, int nvalid, int shift, cx<T>* out, long long pOut, int ldOut, int nstore,
                     const cx<T>* mul = nullptr) {
  if constexpr (sizeof(T) == 4) {
    if (shift == 0 && tr.fR0 && fx3_supported(tr.desc.P)) {
      for (int p0 = 0; p0 < nplanes; p0 += kMaxPlanes) {
        const int np = std::min(kMaxPlanes, nplanes - p0);
        ECC_HIP(launch_fx_cols(st, tr.desc.P, dir, np, in + p0 * pIn, pIn, ldIn, ncols, nvalid, out + p0 * pOut,
                               pOut, ldOut, nstore, tr.fx(), mul));
      }
      return ECC_OK;
    }
  }
  const ColCfg cc = col_config(tr, kColLgB, sizeof(cx<T>), kColThreads);
  ECC_TRY(check_col(cc, tr, sizeof(cx<T>)));
  for (int p0 = 0; p0 < nplanes; p0 += kMaxPlanes) {
    const int np = std::min(kMaxPlanes, nplanes - p0);
    ECC_HIP((launch_fft_cols<T>(st, cc, np, dir, in + p0 * pIn, pIn, ldIn, ncols, nvalid, shift, out + p0 * pOut,
                                pOut, ldOut, nstore, 0, tr.desc, sizeof(T) == 8 ? (const cx<T>*)tr.d() : (const cx<T>*)tr.f(),
                                mul)));
  }
  return ECC_OK;
}

// Full-size buffers are [..][Pz][Py][Lx]: rows padded to Lx = Px rounded up to 16
// complex values (128 bytes), so that every 16-column block of the column passes starts
// on a cache line in every row; V = Pz Py Lx is the stored size, Pz Py Px the transform's.
struct Geo3 {
  int nz, ny, nx, Pz, Py, Px, Lx;
  long long V;
  const Transform *Tz, *Ty, *Tx;
};

ecc_status geometry3(ecc_context ctx, int R, int nz, int ny, int nx, Geo3& g) {
  g.nz = nz;
  g.ny = ny;
  g.nx = nx;
  // >= n + R (zero boundary), >= 2R + 1 (the filter window does not wrap onto itself)
  g.Pz = next_smooth7(std::max({nz + R, 2 * R + 1, 8}));
  g.Py = next_smooth7(std::max({ny + R, 2 * R + 1, 8}));
  g.Px = next_smooth7(std::max({nx + R, 2 * R + 1, 8}));
  g.Lx = (g.Px + 15) & ~15;
  g.V = (long long)g.Pz * g.Py * g.Lx;
  ECC_HIP(get_transform(ctx, g.Pz, &g.Tz));
  ECC_HIP(get_transform(ctx, g.Py, &g.Ty));
  ECC_HIP(get_transform(ctx, g.Px, &g.Tx));
  return ECC_OK;
}

// Spectra of the components on the Pz x Py x Px grid (float64, rounded once): component
// c placed with offset q at q mod P; correlation: sum_q C(q) e^{+i w q} (the transform of
// C(-q)), convolution: sum_q C(q) e^{-i w q}. Built in chunks of components. partial:
// only the x and y transforms, the S planes of z offsets j - R kept as they are
// ([c][S][Py][Lx]; the z pass forms each column's transform on chip), 1/9 of the bytes
// at 128^3 with a 15^3 filter.
ecc_status volume_spectra(ecc_volume_plan plan, int op, const Geo3& g, bool partial, hipStream_t st,
                          const cx<float>** out) {
  std::lock_guard<std::mutex> lk(plan->mu);
  const auto key = std::make_tuple(op * 2 + (partial ? 1 : 0), g.Pz, g.Py, g.Px);
  auto it = plan->spectra.find(key);
  if (it != plan->spectra.end()) {
    *out = it->second->as<cx<float>>();
    return ECC_OK;
  }
  const int S = plan->S, R = plan->R, U = plan->U;
  const int dir = op == ECC_CORRELATION ? +1 : -1;
  const long long per = partial ? (long long)S * g.Py * g.Lx : g.V;   // stored values per component
  auto buf = std::make_unique<DevBuf>();
  ECC_HIP(buf->ensure((size_t)U * per * sizeof(cx<float>)));
  const int chunk = (int)std::max<long long>(1, std::min<long long>(U, (512LL << 20) / (g.V * 16)));
  DevBuf t1, t2, s64;
  ECC_HIP(t1.ensure((size_t)chunk * S * S * g.Lx * sizeof(cx<double>)));
  ECC_HIP(t2.ensure((size_t)chunk * S * g.Py * g.Lx * sizeof(cx<double>)));
  const int PyLx = g.Py * g.Lx;
  if (!partial) ECC_HIP(s64.ensure((size_t)chunk * g.V * sizeof(cx<double>)));
  const long long S3 = (long long)S * S * S;
  for (int c0 = 0; c0 < U; c0 += chunk) {
    const int nc = std::min(chunk, U - c0);
    const cx<double>* src = plan->comps64.as<cx<double>>() + c0 * S3;
    ECC_TRY((rows_pass<double>(st, *g.Tx, nc * S, dir, src, (long long)S * S, S, S, S, -R, t1.as<cx<double>>(),
                               (long long)S * g.Lx, g.Lx, g.Px)));
    ECC_TRY((cols_pass<double>(st, *g.Ty, nc * S, dir, t1.as<cx<double>>(), (long long)S * g.Lx, g.Lx, g.Px, S, -R,
                               t2.as<cx<double>>(), (long long)PyLx, g.Lx, g.Py)));
    if (partial) {
      ECC_HIP(launch_d2f(st, t2.as<cx<double>>(), buf->as<cx<float>>() + (long long)c0 * per, (long long)nc * per));
      continue;
    }
    ECC_TRY((cols_pass<double>(st, *g.Tz, nc, dir, t2.as<cx<double>>(), (long long)S * PyLx, PyLx, PyLx, S, -R,
                               s64.as<cx<double>>(), g.V, PyLx, g.Pz)));
    ECC_HIP(launch_d2f(st, s64.as<cx<double>>(), buf->as<cx<float>>() + (long long)c0 * g.V, (long long)nc * g.V));
  }
  ECC_HIP(hipStreamSynchronize(st));   // temporaries are freed on return
  *out = buf->as<cx<float>>();
  plan->spectra[key] = std::move(buf);
  return ECC_OK;
}

size_t ws_volume(int U, const Geo3& g) { return ((size_t)2 * U + 1) * (size_t)g.V * sizeof(cx<float>); }

}  // namespace

extern "C" {

ecc_status ecc_volume_plan_create(ecc_context ctx, const float* filter, int S, int K, void* stream,
                                  ecc_volume_plan* out) {
  ECC_REQ(ctx && filter && out, "NULL argument");
  *out = nullptr;
  ECC_REQ(S >= 3 && S <= kMaxSteerS && S % 2 == 1, "filter side must be odd, 3..63");
  ECC_REQ(K >= 0 && K <= kMaxSteerK, "band limit K must be 0..8");
  DeviceGuard dg(ctx->device);
  hipStream_t st = S_(stream);
  auto plan = std::make_unique<ecc_volume_plan_s>();
  plan->ctx = ctx;
  plan->device = ctx->device;
  plan->S = S;
  plan->R = (S - 1) / 2;
  plan->K = K;
  const int R = plan->R;
  for (int l = 0; l <= K; ++l) {
    for (int m = 0; m <= l; ++m) {
      plan->hs.push_back(make_int4(l, 0, m, 0));
      plan->weights.push_back(m == 0 ? 1.f : 2.f);
    }
    for (int mp = 1; mp <= l; ++mp)
      for (int m = -l; m <= l; ++m) {
        plan->hs.push_back(make_int4(l, mp, m, 0));
        plan->weights.push_back(2.f);
      }
  }
  const int U = (int)plan->hs.size();
  plan->U = U;
  // Wigner's coefficients, one per term k of d^l_{m'm}, in half-set order
  std::vector<double> coef;
  for (const int4& h : plan->hs) {
    const int l = h.x, mp = h.y, m = h.z;
    const long double pre = sqrtl(lfact(l + mp) * lfact(l - mp) * lfact(l + m) * lfact(l - m));
    for (int k = std::max(0, m - mp); k <= std::min(l + m, l - mp); ++k) {
      const long double sg = ((mp - m + k) % 2) ? -1.0L : 1.0L;
      coef.push_back((double)(sg * pre / (lfact(l + m - k) * lfact(k) * lfact(mp - m + k) * lfact(l - mp - k))));
    }
  }
  ECC_HIP(plan->coef.ensure(coef.size() * sizeof(double)));
  ECC_HIP(hipMemcpy(plan->coef.p, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice));
  ECC_HIP(plan->d_w.ensure(U * sizeof(float)));
  ECC_HIP(hipMemcpy(plan->d_w.p, plan->weights.data(), U * sizeof(float), hipMemcpyHostToDevice));

  // quadrature: M azimuths, M / 2 Gauss-Legendre polar nodes; every distinct grid radius
  const int M = azimuths(K, R), nt = M / 2;
  plan->M = M;
  std::vector<double> gt, gw;
  gauss_legendre(nt, gt, gw);
  std::vector<int> d2list, rindex(R * R + 1, -1);
  for (int d2 = 1; d2 <= R * R; ++d2) {
    bool ok = false;
    for (int a = 0; a <= R && !ok; ++a)
      for (int b = a; b <= R && !ok; ++b) {
        const int c2 = d2 - a * a - b * b;
        if (c2 < b * b) break;
        const int c = (int)std::lround(std::sqrt((double)c2));
        ok = c * c == c2 && c <= R;
      }
    if (ok) {
      rindex[d2] = (int)d2list.size();
      d2list.push_back(d2);
    }
  }
  const int nr = (int)d2list.size();
  DevBuf d_t, d_wq, d_d2, d_A, d_f, d_hs, d_ri;
  ECC_HIP(d_t.ensure(nt * sizeof(double)));
  ECC_HIP(d_wq.ensure(nt * sizeof(double)));
  ECC_HIP(d_d2.ensure(std::max(1, nr) * sizeof(int)));
  ECC_HIP(d_A.ensure((size_t)std::max(1, nr) * nt * (K + 1) * sizeof(cx<double>)));
  ECC_HIP(d_f.ensure((size_t)std::max(1, nr) * (K + 1) * (2 * K + 1) * sizeof(cx<double>)));
  ECC_HIP(d_hs.ensure(U * sizeof(int4)));
  ECC_HIP(d_ri.ensure(rindex.size() * sizeof(int)));
  ECC_HIP(hipMemcpy(d_t.p, gt.data(), nt * sizeof(double), hipMemcpyHostToDevice));
  ECC_HIP(hipMemcpy(d_wq.p, gw.data(), nt * sizeof(double), hipMemcpyHostToDevice));
  if (nr) ECC_HIP(hipMemcpy(d_d2.p, d2list.data(), nr * sizeof(int), hipMemcpyHostToDevice));
  ECC_HIP(hipMemcpy(d_hs.p, plan->hs.data(), U * sizeof(int4), hipMemcpyHostToDevice));
  ECC_HIP(hipMemcpy(d_ri.p, rindex.data(), rindex.size() * sizeof(int), hipMemcpyHostToDevice));
  const long long S3 = (long long)S * S * S;
  ECC_HIP(plan->comps64.ensure((size_t)U * S3 * sizeof(cx<double>)));
  ECC_HIP(plan->comps32.ensure((size_t)U * S3 * sizeof(cx<float>)));
  if (nr) {
    ECC_HIP(launch_sh_azimuth(st, filter, S, K, M, nt, d_t.as<double>(), nr, d_d2.as<int>(), d_A.as<cx<double>>()));
    ECC_HIP(launch_sh_polar(st, d_A.as<cx<double>>(), nr, nt, K, M, d_t.as<double>(), d_wq.as<double>(),
                            d_f.as<cx<double>>()));
  }
  ECC_HIP(launch_sh_components(st, filter, S, K, U, d_hs.as<int4>(), d_ri.as<int>(), d_f.as<cx<double>>(),
                               plan->comps64.as<cx<double>>()));
  ECC_HIP(launch_d2f(st, plan->comps64.as<cx<double>>(), plan->comps32.as<cx<float>>(), (long long)U * S3));
  ECC_HIP(hipStreamSynchronize(st));
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->vplans.insert(plan.get());
  }
  *out = plan.release();
  return ECC_OK;
}

ecc_status ecc_volume_plan_destroy(ecc_volume_plan plan) {
  if (!plan) return ECC_OK;
  DeviceGuard dg(plan->device);
  (void)hipDeviceSynchronize();
  {
    std::lock_guard<std::mutex> g(plan->ctx->mu);
    plan->ctx->vplans.erase(plan);
  }
  delete plan;
  return ECC_OK;
}

ecc_status ecc_volume_plan_info(ecc_volume_plan plan, int* U, int* M) {
  ECC_REQ(plan, "NULL plan");
  if (U) *U = plan->U;
  if (M) *M = plan->M;
  return ECC_OK;
}

ecc_status ecc_volume_plan_components(ecc_volume_plan plan, float* comps, int* table, float* weights, void* stream) {
  ECC_REQ(plan, "NULL plan");
  DeviceGuard dg(plan->device);
  if (comps) {
    const size_t n = (size_t)plan->U * plan->S * plan->S * plan->S * sizeof(cx<float>);
    ECC_HIP(hipMemcpyAsync(comps, plan->comps32.p, n, hipMemcpyDeviceToDevice, S_(stream)));
    ECC_HIP(hipStreamSynchronize(S_(stream)));
  }
  for (int c = 0; c < plan->U; ++c) {
    if (table) {
      table[3 * c] = plan->hs[c].x;
      table[3 * c + 1] = plan->hs[c].y;
      table[3 * c + 2] = plan->hs[c].z;
    }
    if (weights) weights[c] = plan->weights[c];
  }
  return ECC_OK;
}

ecc_status ecc_volume_workspace_size(ecc_context ctx, ecc_volume_plan plan, int nz, int ny, int nx, size_t* bytes) {
  ECC_REQ(ctx && plan && bytes, "NULL argument");
  ECC_REQ(nz >= 1 && ny >= 1 && nx >= 1, "empty volume");
  DeviceGuard dg(ctx->device);
  Geo3 g{};
  ECC_TRY(geometry3(ctx, plan->R, nz, ny, nx, g));
  *bytes = ws_volume(plan->U, g);
  return ECC_OK;
}

ecc_status ecc_extended_3d(ecc_context ctx, ecc_op op, ecc_volume_plan plan, int nz, int ny, int nx,
                           const float* signal, const float* alpha, const float* beta, const float* gamma,
                           float* out, void* stream) {
  ECC_REQ(ctx && plan, "NULL context or plan");
  ECC_REQ(plan->ctx == ctx, "plan belongs to another context");
  ECC_REQ(op == ECC_CORRELATION || op == ECC_CONVOLUTION, "unknown op");
  ECC_REQ(signal && alpha && beta && gamma && out, "NULL volume pointer");
  ECC_REQ(nz >= 1 && ny >= 1 && nx >= 1, "empty volume");
  ECC_REQ((long long)nz * ny * nx <= (1LL << 31) - 1, "volume too large");
  const long long nv = (long long)nz * ny * nx;
  const size_t bo = (size_t)nv * sizeof(float);
  ECC_REQ(!overlaps(out, bo, signal, bo) && !overlaps(out, bo, alpha, bo) && !overlaps(out, bo, beta, bo) &&
              !overlaps(out, bo, gamma, bo),
          "out aliases an input");
  DeviceGuard dg(ctx->device);
  hipStream_t st = S_(stream);
  Geo3 g{};
  ECC_TRY(geometry3(ctx, plan->R, nz, ny, nx, g));
  ECC_REQ((long long)g.Pz * g.Py * g.Lx <= (1LL << 31) - 1, "volume too large");
  // with the compiled z transform the spectra stay partial (the z pass forms them)
  const bool partial = g.Tz->fR0 && fx3_supported(g.Pz);
  const cx<float>* Sp = nullptr;
  ECC_TRY(volume_spectra(plan, op, g, partial, st, &Sp));
  const int S = plan->S;
  const long long planeSp = partial ? (long long)S * g.Py * g.Lx : g.V;
  WsUse wu(ctx, st);
  const int U = plan->U;
  ECC_HIP(ctx->ws.ensure(ws_volume(U, g)));
  cx<float>* A = ctx->ws.as<cx<float>>();
  cx<float>* Z = A + g.V;
  cx<float>* W = Z + (long long)U * g.V;
  const int PyLx = g.Py * g.Lx, Lx = g.Lx;
  const long long plane = (long long)PyLx;
  const float scale = (float)(1.0 / ((double)g.Pz * g.Py * g.Px));
  if (op == ECC_CORRELATION) {
    // H -> spectrum A (x, y, z passes), products with every component's spectrum
    ECC_HIP(launch_real_to_cx(st, signal, Z, nv));
    ECC_TRY((rows_pass<float>(st, *g.Tx, nz, -1, Z, (long long)ny * nx, nx, ny, nx, 0, W, plane, Lx, g.Px)));
    ECC_TRY((cols_pass<float>(st, *g.Ty, nz, -1, W, plane, Lx, g.Px, ny, 0, Z, plane, Lx, g.Py)));
    ECC_TRY((cols_pass<float>(st, *g.Tz, 1, -1, Z, 0, PyLx, PyLx, nz, 0, A, 0, PyLx, g.Pz)));
    // inverse transforms of the products A Sp_c (formed as the first pass loads them), only
    // the output voxels kept
    if (partial)
      ECC_HIP(launch_fx_cols_corr(st, g.Pz, U, Sp, planeSp, PyLx, PyLx, S, plan->R, A, W, (long long)nz * PyLx, nz,
                                  g.Tz->fx()));
    else
      ECC_TRY((cols_pass<float>(st, *g.Tz, U, +1, Sp, g.V, PyLx, PyLx, g.Pz, 0, W, (long long)nz * PyLx, PyLx, nz,
                                A)));
    ECC_TRY((cols_pass<float>(st, *g.Ty, U * nz, +1, W, plane, Lx, g.Px, g.Py, 0, Z, (long long)ny * Lx, Lx, ny)));
    if (g.Tx->fR0 && fx_rows_wigner_supported(g.Px, plan->K, nx)) {
      // last pass and the Wigner-D combination in one kernel (no component volumes stored)
      ECC_HIP(launch_fx_rows_wigner(st, g.Px, plan->K, Z, (long long)nz * ny * Lx, Lx, nz * ny, g.Px, nx, alpha,
                                    beta, gamma, plan->coef.as<double>(), plan->d_w.as<float>(), out, scale,
                                    g.Tx->fx()));
    } else {
      ECC_TRY((rows_pass<float>(st, *g.Tx, U, +1, Z, (long long)nz * ny * Lx, Lx, nz * ny, g.Px, 0, W, nv, nx, nx)));
      // Wigner-D combination per voxel
      ECC_HIP(launch_wigner_voxels(st, plan->K, 0, alpha, beta, gamma, nv, plan->coef.as<double>(),
                                   plan->d_w.as<float>(), W, nullptr, out, nullptr, scale));
    }
  } else {
    // modulated signals H D_c, their spectra, the weighted sum of products, one inverse
    ECC_HIP(launch_wigner_voxels(st, plan->K, 1, alpha, beta, gamma, nv, plan->coef.as<double>(),
                                 plan->d_w.as<float>(), nullptr, signal, nullptr, Z, 1.0f));
    ECC_TRY((rows_pass<float>(st, *g.Tx, U * nz, -1, Z, (long long)ny * nx, nx, ny, nx, 0, W, plane, Lx, g.Px)));
    ECC_TRY((cols_pass<float>(st, *g.Ty, U * nz, -1, W, plane, Lx, g.Px, ny, 0, Z, plane, Lx, g.Py)));
    if (partial) {
      // z pass and the weighted product sum in one kernel (each spectrum column formed on
      // chip; components summed in registers, in four groups whose partial sums W holds,
      // then added in order)
      ECC_HIP(launch_fx_cols_accum(st, g.Pz, U, Z, (long long)nz * PyLx, PyLx, PyLx, nz, Sp, planeSp, S, plan->R,
                                   plan->d_w.as<float>(), 4, W, g.V, A, PyLx, g.Tz->fx()));
    } else {
      ECC_TRY((cols_pass<float>(st, *g.Tz, U, -1, Z, (long long)nz * PyLx, PyLx, PyLx, nz, 0, W, g.V, PyLx, g.Pz)));
      ECC_HIP(launch_spec_accumulate(st, W, Sp, plan->d_w.as<float>(), g.V, U, A));
    }
    ECC_TRY((cols_pass<float>(st, *g.Tz, 1, +1, A, 0, PyLx, PyLx, g.Pz, 0, Z, 0, PyLx, nz)));
    ECC_TRY((cols_pass<float>(st, *g.Ty, nz, +1, Z, plane, Lx, g.Px, g.Py, 0, W, (long long)ny * Lx, Lx, ny)));
    ECC_TRY((rows_pass<float>(st, *g.Tx, 1, +1, W, 0, Lx, nz * ny, g.Px, 0, Z, 0, nx, nx)));
    ECC_HIP(launch_real_part(st, Z, out, nv, scale));
  }
  return ECC_OK;
}

}  // extern "C"
