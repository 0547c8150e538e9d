// C-ABI of libecc: validation, plan construction, and the launch sequences of the
// correlation / convolution / matching / smoothing / adjoint paths.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "api_common.hpp"

using namespace ecc;

thread_local std::string g_err;

namespace ecc {
ecc_status fail(ecc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
}  // namespace ecc

namespace {

int tune_fft_size(ecc_context ctx, int n, int Pmin);
bool two_pass_size_ok(ecc_context ctx, int P);
ColCfg corr_col_config(const Transform& t);

// FFT size of the two-pass form for an image side n and filter radius R: the smallest
// 7-smooth size >= max(n + R, 2R + 1, 16) (at least 16: every transform then has two or
// more passes, and zero padding beyond n + R changes nothing in the result; at least
// 2R + 1: the filter window is placed without wrapping onto itself) that every two-pass
// kernel takes (two_pass_size_ok; a size with too many butterflies per pass is passed
// over for the next one, up to 4096). With the autotuner on, the fastest of the 7-smooth
// sizes up to 1/8 above it (tune_fft_size), chosen once per context and side.
int fft_size_for(ecc_context ctx, int n, int R) {
  int Pmin = next_smooth7(std::max(std::max(n + R, 2 * R + 1), 16));
  for (int P = Pmin; P <= 4096; P = next_smooth7(P + 1))
    if (two_pass_size_ok(ctx, P)) {
      Pmin = P;
      break;
    }
  const std::string key = std::to_string(n) + ":" + std::to_string(R);
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) return it->second;
  }
  if (!ctx->autotune) return Pmin;
  const int P = tune_fft_size(ctx, n, Pmin);   // (launches kernels: outside the lock)
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->tuned.emplace(key, P);
  return ctx->tuned[key];
}

}  // namespace
namespace ecc {
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}
}  // namespace ecc
namespace {


// complex row pitch rounded up to 16 elements (128 bytes)
inline int pitch16(int n) { return (n + 15) & ~15; }

// ---- bytes of context workspace each path uses; the call sites and ecc_workspace_size
// both take them from here
// two-pass correlation stack: row spectra ny x W', signal spectrum Py x W', and two
// (direct, mirror) planes per component, W' = pitch16(Px / 2 + 1)
size_t ws_corr_stack(int batch, int ny, int Py, int Px, int U) {
  const size_t ldW = (size_t)pitch16(Px / 2 + 1);
  return (size_t)batch * ((size_t)ny * ldW + (size_t)Py * ldW + 2 * (size_t)ny * ldW * U) * sizeof(cx<float>);
}
// component groups of the two-pass convolution's column kernel: with fewer column
// blocks than two per CU (a small batch of narrow images) the components are split so
// that about 2048 workgroups run; the groups' partial sums are then added by a second
// kernel. (With two or more blocks per CU the column transforms' LDS already limits the
// workgroups per CU, and the split only adds the partial planes' traffic.)
int conv_col_groups(int batch, int Px, int U) {
  const long long blocks = (long long)((Px + 3) / 4) * batch;
  if (blocks >= 512) return 1;
  const long long g = (2048 + blocks - 1) / blocks;
  return (int)std::max(1LL, std::min<long long>(g, std::min(U, 16)));
}
// two-pass convolution: modulated row spectra (unless saved by the caller), the
// column-summed plane per signal, and the component groups' partial Py x Px planes
size_t ws_conv_two_pass(int batch, int ny, int Py, int Px, int U, int nsig, bool saved) {
  const size_t plane = (size_t)ny * Px;
  const int G = conv_col_groups(batch, Px, U);
  const size_t part = G > 1 ? (size_t)G * batch * nsig * Py * Px : 0;
  return ((saved ? 0 : (size_t)batch * nsig * U * plane) + (size_t)batch * nsig * plane + part) * sizeof(cx<float>);
}
// tiled matching: the component stack, U planes of ny x nx
size_t ws_match_tiled(int ny, int nx, int U) { return (size_t)stack_pitch((long long)ny * nx) * U * sizeof(cx<float>); }
// on-chip filter gradient: per-block lag sums (256-byte aligned) + the reduction's scratch
size_t ws_gradf_parts(long long nblk, int U, int Sz) {
  return ((size_t)nblk * U * Sz * Sz * sizeof(cx<float>) + 255) / 256 * 256;
}
// two-pass filter gradient: row and full spectra of the output gradient, the product
// planes, the column-transformed lags, the lag windows and (unless saved) the stack
size_t ws_gradf_two_pass(int batch, int ny, int Py, int Px, int U, int Sz, bool saved) {
  const size_t W = (size_t)(Px / 2 + 1);
  size_t n = (size_t)batch * ((size_t)ny * W + (size_t)Py * W) + (size_t)U * Py * Px + (size_t)U * Sz * Px +
             (size_t)U * Sz * Sz;
  if (!saved) n += (size_t)batch * U * ny * Px;
  return n * sizeof(cx<float>);
}

ecc_status check_cfg_row(const RowCfg& c, const Transform& t, size_t elem, const char* what) {
  if (c.NB < 0 || c.EPX < 0 || lds_rows(c, t.desc, elem) > kMaxLds)
    return fail(ECC_ERR_UNSUPPORTED, std::string("transform too long for the ") + what + " kernel");
  return ECC_OK;
}
ecc_status check_cfg_col(const ColCfg& c, const Transform& t, size_t elem, const char* what, bool need_ept) {
  if (c.NB < 0 || (need_ept && c.EPT < 0) || lds_cols(c, t.desc, elem) > kMaxLds)
    return fail(ECC_ERR_UNSUPPORTED, std::string("transform too long for the ") + what + " kernel");
  return ECC_OK;
}


// Whether every two-pass kernel takes transforms of length P: rows with at most 256
// threads per line (the correlation's combined inverse row kernel runs two per
// workgroup), the column kernels' configurations.
bool two_pass_size_ok(ecc_context ctx, int P) {
  const Transform* T = nullptr;
  if (get_transform(ctx, P, &T) != hipSuccess) return false;
  const RowCfg r = row_config(*T, P, sizeof(cx<float>));
  const ColCfg c2 = col_config(*T, 2, sizeof(cx<float>), 512);
  return r.TF <= 256 && r.NB > 0 && r.EPX > 0 && lds_rows(r, T->desc, sizeof(cx<float>)) <= kMaxLds &&
         c2.NB > 0 && c2.EPT > 0 && lds_cols(c2, T->desc, sizeof(cx<float>)) <= kMaxLds &&
         corr_col_config(*T).NB > 0;
}

// Launch shape of the two-pass correlation's component column kernel (1024 threads): it
// takes at most two butterflies and 16 rows per thread, so narrower column blocks are
// tried when 4-column blocks exceed that (long transforms of small radices); NB = -1 if
// no block width fits.
ColCfg corr_col_config(const Transform& t) {
  ColCfg c{};
  for (int lgB = 2; lgB >= 0; --lgB) {
    c = col_config(t, lgB, sizeof(cx<float>), 1024);
    const int TF = c.nthr >> c.lgB;
    if (c.NB > 0 && c.NB <= 2 && (t.desc.P + TF - 1) / TF <= 16 &&
        check_cfg_col(c, t, sizeof(cx<float>), "column", true) == ECC_OK)
      return c;
  }
  c.NB = -1;
  return c;
}

// The candidates of fft_size_for are timed as the two-pass correlation's own kernels on up
// to 512 rows of an n-wide signal: the forward row and column transforms of the signal and
// the inverse row pass of four components with the per-pixel combination (the dominant
// stage, which runs on a compiled schedule for some lengths), best of three after one
// warm-up run, on a private stream. A size the two-pass calls would refuse is skipped;
// any failure keeps the smallest size.
int tune_fft_size(ecc_context ctx, int n, int Pmin) {
  std::vector<int> cand{Pmin};
  for (int P = next_smooth7(Pmin + 1); (long long)P * 8 <= (long long)Pmin * 9 && cand.size() < 4;
       P = next_smooth7(P + 1))
    cand.push_back(P);
  if (cand.size() == 1) return Pmin;
  DeviceGuard dg(ctx->device);
  constexpr int Ucal = 4;
  const int rows = std::min(n, 512);
  const int Pmax = cand.back(), ldW = (Pmax / 2 + 1 + 15) & ~15;
  const long long pTk = 2LL * rows * ldW;
  DevBuf h, a, hh, tk, yb, wb;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) e = h.ensure((size_t)rows * n * sizeof(float));
  if (e == hipSuccess) e = a.ensure((size_t)rows * ldW * sizeof(cx<float>));
  if (e == hipSuccess) e = hh.ensure((size_t)Pmax * ldW * sizeof(cx<float>));
  if (e == hipSuccess) e = tk.ensure((size_t)Ucal * pTk * sizeof(cx<float>));
  if (e == hipSuccess) e = yb.ensure((size_t)rows * n * sizeof(float));
  if (e == hipSuccess) e = wb.ensure(Ucal * sizeof(float));
  if (e == hipSuccess) e = hipMemsetAsync(h.p, 0, (size_t)rows * n * sizeof(float), st);
  if (e == hipSuccess) e = hipMemsetAsync(tk.p, 0, (size_t)Ucal * pTk * sizeof(cx<float>), st);
  if (e == hipSuccess) e = hipMemsetAsync(wb.p, 0, Ucal * sizeof(float), st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  Field fl{h.as<float>(), 0, n, 0, 1.0, 0.0};   // the zero signal doubles as the angle field
  int best = Pmin;
  double best_ms = 1e30;
  for (int P : cand) {
    if (e != hipSuccess) break;
    const Transform* T = nullptr;
    if (get_transform(ctx, P, &T) != hipSuccess) continue;
    const int W = P / 2 + 1;
    const RowCfg r1 = row_config(*T, P, sizeof(cx<float>));
    const ColCfg c2 = col_config(*T, 2, sizeof(cx<float>), 512);
    const ColCfg c3 = corr_col_config(*T);   // a size the two-pass calls would refuse is no candidate
    RowCfg r4 = row_config(*T, n, sizeof(cx<float>));
    r4.B = 2;
    if (r4.TF > 256 || check_cfg_row(r1, *T, sizeof(cx<float>), "row") != ECC_OK ||
        check_cfg_col(c2, *T, sizeof(cx<float>), "column", true) != ECC_OK ||
        check_cfg_col(c3, *T, sizeof(cx<float>), "column", true) != ECC_OK ||
        (T->fR0 <= 0 && check_cfg_row(r4, *T, sizeof(cx<float>), "row") != ECC_OK))
      continue;
    double ms_min = 1e30;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
      e = hipEventRecord(e0, st);
      if (e == hipSuccess)
        e = launch_rows_r2c(st, r1, 1, h.as<float>(), 0, n, a.as<cx<float>>(), 0, ldW, rows, n, W, T->desc,
                            T->f());
      if (e == hipSuccess)
        e = launch_cols_fwd(st, c2, 1, a.as<cx<float>>(), 0, ldW, rows, W, hh.as<cx<float>>(), 0, ldW, T->desc,
                            T->f());
      if (e == hipSuccess) {
        if (T->fR0 > 0)
          e = launch_corr_rows_fixed(st, 4, 1, tk.as<cx<float>>(), pTk, Ucal * pTk, ldW, fl, yb.as<float>(), 0, n,
                                     rows, n, Ucal, wb.as<float>(), 1.0f, nullptr, nullptr, 0, 0, 1.0f, 0, 0, P,
                                     T->fx());
        else
          e = launch_corr_rows(st, r4, 1, tk.as<cx<float>>(), pTk, Ucal * pTk, ldW, fl, yb.as<float>(), 0, n, rows,
                               n, Ucal, wb.as<float>(), 1.0f, nullptr, nullptr, 0, 0, 1.0f, 0, 0, T->desc, T->f());
      }
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && rep > 0) ms_min = std::min(ms_min, (double)ms);
    }
    if (e == hipSuccess && ms_min < best_ms) {
      best_ms = ms_min;
      best = P;
    }
  }
  if (st) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e == hipSuccess ? best : Pmin;
}

// records stage event i of the measurement hook, if set
inline hipError_t mark_event(ecc_context ctx, int i, hipStream_t st) {
  if (i < (int)ctx->stage_events.size()) return hipEventRecord(ctx->stage_events[i], st);
  return hipSuccess;
}
#define mark(ctx, i, st) ECC_HIP(mark_event(ctx, i, st))

// Filter spectra Fh_k = FFT2(F_k placed with its centre at (0, 0)) on a Py x Px grid,
// computed in float64 and rounded to float32. Symmetric plans keep columns [0, W).
ecc_status get_spectrum(ecc_filter_plan plan, int Py, int Px, hipStream_t st, const Spectrum** out) {
  std::lock_guard<std::mutex> g(plan->mu);
  auto key = std::make_pair(Py, Px);
  auto it = plan->spectra.find(key);
  if (it != plan->spectra.end()) {
    *out = it->second.get();
    return ECC_OK;
  }
  const Transform *Ty = nullptr, *Tx = nullptr;
  ECC_HIP(get_transform(plan->ctx, Py, &Ty));
  ECC_HIP(get_transform(plan->ctx, Px, &Tx));
  auto sp = std::make_unique<Spectrum>();
  sp->Py = Py;
  sp->Px = Px;
  sp->full = plan->symmetric ? 0 : 1;
  const int W = Px / 2 + 1;
  const int Wst = sp->full ? Px : W;
  const int ld = pitch16(Wst);   // rows start on 128-byte boundaries
  sp->ld = ld;
  const int U = plan->U, Sz = plan->S, R = plan->R;
  DevBuf tmp, spec64;
  ECC_HIP(tmp.ensure((size_t)U * Sz * ld * sizeof(cx<double>)));
  ECC_HIP(spec64.ensure((size_t)U * Py * ld * sizeof(cx<double>)));
  ECC_HIP(sp->buf.ensure((size_t)U * Py * ld * sizeof(cx<float>)));
  ECC_HIP(hipMemsetAsync(spec64.p, 0, (size_t)U * Py * ld * sizeof(cx<double>), st));
  // float64 transforms: 256 threads per line, or 512 for lengths whose passes have more
  // butterflies than 256 threads take (about 3000 and above)
  RowCfg rc = row_config(*Tx, Px, sizeof(cx<double>));
  if (rc.NB < 0 || rc.EPX < 0) rc = row_config(*Tx, Px, sizeof(cx<double>), 512);
  ColCfg cc = col_config(*Ty, 2, sizeof(cx<double>), 256);
  if (cc.NB < 0) cc = col_config(*Ty, 2, sizeof(cx<double>), 512);
  ECC_TRY(check_cfg_row(rc, *Tx, sizeof(cx<double>), "filter row"));
  ECC_TRY(check_cfg_col(cc, *Ty, sizeof(cx<double>), "filter column", false));
  ECC_HIP((launch_fft_rows<double>(st, rc, U, -1, plan->comps64.as<cx<double>>(), (long long)Sz * Sz, Sz,
                                   Sz, Sz, -R, tmp.as<cx<double>>(), (long long)Sz * ld, ld, Wst, 0,
                                   Tx->desc, Tx->d())));
  ECC_HIP((launch_fft_cols<double>(st, cc, U, -1, tmp.as<cx<double>>(), (long long)Sz * ld, ld, Wst,
                                   Sz, -R, spec64.as<cx<double>>(), (long long)Py * ld, ld, Py, 0,
                                   Ty->desc, Ty->d())));
  ECC_HIP(launch_d2f(st, spec64.as<cx<double>>(), sp->buf.as<cx<float>>(), (long long)U * Py * ld));
  ECC_HIP(hipStreamSynchronize(st));   // temporaries are freed on return
  *out = sp.get();
  plan->spectra[key] = std::move(sp);
  return ECC_OK;
}

}  // namespace
namespace ecc {
// Block spectra for the tiled path: FFT_N x N(F_k placed with its window corner at
// (0, 0)), float64 then rounded, full N x N planes (no symmetry assumed).
bool rotation_parity(ecc_filter_plan plan) {
  if (plan->group != ECC_GROUP_ROTATION || !plan->symmetric || (int)plan->parity.size() != plan->U) return false;
  for (int k = 0; k < plan->U; ++k)
    if (plan->parity[k] != ((k % 2) ? -1.f : 1.f)) return false;
  return true;
}

const Spectrum* find_tile_spectrum(ecc_filter_plan plan, int N, int mode) {
  std::lock_guard<std::mutex> g(plan->mu);
  auto it = plan->tile_spectra.find(mode * 1000 + N);
  return it == plan->tile_spectra.end() ? nullptr : it->second.get();
}

ecc_status get_tile_spectrum(ecc_filter_plan plan, int N, hipStream_t st, const Spectrum** out, int mode) {
  std::lock_guard<std::mutex> g(plan->mu);
  const bool conv = mode == SPEC_CONV;
  const int key = mode * 1000 + N;
  auto it = plan->tile_spectra.find(key);
  if (it != plan->tile_spectra.end()) {
    *out = it->second.get();
    return ECC_OK;
  }
  const Transform* Tn = nullptr;
  ECC_HIP(get_transform(plan->ctx, N, &Tn));
  auto sp = std::make_unique<Spectrum>();
  sp->Py = sp->Px = N;
  sp->full = 1;
  const int U = plan->U, Sz = plan->S;
  // correlation: F_k with its window corner at (0, 0), planes of N x N; convolution:
  // offset x at x - R, planes of tconv_plane(N) values with row pitch N + 1
  const bool ratio = mode == SPEC_RATIO;
  if (ratio && (!plan->symmetric || (int)plan->parity.size() != U))
    return fail(ECC_ERR_INTERNAL, "ratio spectra need components with parity");
  const bool centred = mode == SPEC_CENTRED || mode == SPEC_CENTRED_CONJ || ratio;
  const bool cconj = mode == SPEC_CORR_CONJ || mode == SPEC_CENTRED_CONJ;
  const int shift = conv ? -2 * plan->R : centred ? -plan->R : 0;
  sp->ld = conv ? tconv_pitch(N) : N;
  const long long plane = conv ? (long long)tconv_plane(N) : (long long)N * N;
  DevBuf tmp, spec64, ccomps;
  ECC_HIP(tmp.ensure((size_t)U * Sz * N * sizeof(cx<double>)));
  const cx<double>* src = plan->comps64.as<cx<double>>();
  if (cconj) {
    ECC_HIP(ccomps.ensure((size_t)U * Sz * Sz * sizeof(cx<double>)));
    ECC_HIP(launch_conj_d(st, src, ccomps.as<cx<double>>(), (long long)U * Sz * Sz));
    src = ccomps.as<cx<double>>();
  }
  ECC_HIP(spec64.ensure((size_t)U * plane * sizeof(cx<double>)));
  ECC_HIP(sp->buf.ensure((size_t)U * plane * sizeof(cx<float>)));
  if (conv) ECC_HIP(hipMemsetAsync(spec64.p, 0, (size_t)U * plane * sizeof(cx<double>), st));
  RowCfg rc = row_config(*Tn, N, sizeof(cx<double>));
  ColCfg cc = col_config(*Tn, 2, sizeof(cx<double>), 256);
  ECC_TRY(check_cfg_row(rc, *Tn, sizeof(cx<double>), "filter row"));
  ECC_TRY(check_cfg_col(cc, *Tn, sizeof(cx<double>), "filter column", false));
  ECC_HIP((launch_fft_rows<double>(st, rc, U, -1, src, (long long)Sz * Sz, Sz,
                                   Sz, Sz, shift, tmp.as<cx<double>>(), (long long)Sz * N, N, N, 0,
                                   Tn->desc, Tn->d())));
  ECC_HIP((launch_fft_cols<double>(st, cc, U, -1, tmp.as<cx<double>>(), (long long)Sz * N, N, N, Sz, shift,
                                   spec64.as<cx<double>>(), plane, sp->ld, N, 0, Tn->desc, Tn->d())));
  if (ratio)
    ECC_HIP(launch_ratio_spectra(st, spec64.as<cx<double>>(), U, N, plan->d_weights.as<float>(),
                                 plan->d_parity.as<float>(), sp->buf.as<float2>()));
  else
    ECC_HIP(launch_d2f(st, spec64.as<cx<double>>(), sp->buf.as<cx<float>>(), (long long)U * plane));
  ECC_HIP(hipStreamSynchronize(st));
  *out = sp.get();
  plan->tile_spectra[key] = std::move(sp);
  return ECC_OK;
}
}  // namespace ecc
namespace {





ecc_status finish_plan(ecc_filter_plan p, hipStream_t st) {
  const size_t n = (size_t)p->U * p->S * p->S;
  ECC_HIP(p->comps32.ensure(n * sizeof(cx<float>)));
  ECC_HIP(launch_d2f(st, p->comps64.as<cx<double>>(), p->comps32.as<cx<float>>(), (long long)n));
  ECC_HIP(p->d_weights.ensure(p->U * sizeof(float)));
  ECC_HIP(hipMemcpyAsync(p->d_weights.p, p->weights.data(), p->U * sizeof(float), hipMemcpyHostToDevice, st));
  if (p->symmetric) {
    ECC_HIP(p->d_parity.ensure(p->U * sizeof(float)));
    ECC_HIP(hipMemcpyAsync(p->d_parity.p, p->parity.data(), p->U * sizeof(float), hipMemcpyHostToDevice, st));
  }
  ECC_HIP(hipStreamSynchronize(st));
  return ECC_OK;
}

struct ScaleSetup {
  double sigma0, smin, smax, pf, u_lo, u_hi, L;
  int n, R;
};

ecc_status scale_setup(const ecc_group_params* gp, ScaleSetup& s) {
  s.sigma0 = (gp && gp->sigma0 > 0) ? gp->sigma0 : 1.0;
  s.smin = (gp && gp->scale_min > 0) ? gp->scale_min : 1.0;
  s.smax = (gp && gp->scale_max > 0) ? gp->scale_max : 8.0;
  s.n = (gp && gp->scale_components > 0) ? gp->scale_components : 24;
  s.pf = (gp && gp->scale_period_factor > 0) ? gp->scale_period_factor : 1.5;
  ECC_REQ(s.smax >= s.smin, "scale_max must be >= scale_min");
  ECC_REQ(s.n >= 2 && s.n <= 512, "scale_components must be in [2, 512]");
  ECC_REQ(s.pf > 1.0, "scale_period_factor must exceed 1");
  s.R = (int)std::ceil(4.0 * s.sigma0 * s.smax - 1e-12);
  ECC_REQ(s.R >= 1 && s.R <= 127, "scaled filter radius ceil(4 sigma0 scale_max) must be in [1, 127]");
  s.u_lo = -std::log(s.smax);
  s.u_hi = std::log((double)s.R) - std::log(s.smin);
  s.L = s.pf * (s.u_hi - s.u_lo);
  return ECC_OK;
}

void scale_plan_fields(ecc_filter_plan p, const ScaleSetup& s) {
  p->U = s.n / 2 + 1;
  p->K = p->U - 1;
  p->R = s.R;
  p->S = 2 * s.R + 1;
  p->M = 0;
  p->weights.assign(p->U, 2.f);
  p->weights[0] = 1.f;
  if (s.n % 2 == 0) p->weights[p->U - 1] = 1.f;
  p->field_mul = 2.0 * 3.14159265358979323846 / s.L;
  p->log_mode = 1;
  p->sig_norm = 1;
}

}  // namespace

// =====================================================================================
extern "C" {

const char* ecc_status_string(ecc_status s) {
  switch (s) {
    case ECC_OK: return "ok";
    case ECC_ERR_INVALID_ARGUMENT: return "invalid argument";
    case ECC_ERR_UNSUPPORTED: return "unsupported";
    case ECC_ERR_OUT_OF_MEMORY: return "out of memory";
    case ECC_ERR_HIP: return "HIP error";
    case ECC_ERR_PLAN_MISMATCH: return "plan mismatch";
    case ECC_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* ecc_last_error(ecc_context) { return g_err.c_str(); }

ecc_status ecc_create(int hip_device, ecc_context* out) {
  ECC_REQ(out != nullptr, "out is NULL");
  *out = nullptr;
  int n = 0;
  ECC_HIP(hipGetDeviceCount(&n));
  ECC_REQ(hip_device >= 0 && hip_device < n, "no such HIP device");
  DeviceGuard dg(hip_device);
  static std::once_flag once;
  static hipError_t prep = hipSuccess;
  std::call_once(once, [] { prep = prepare_kernels(); });
  ECC_HIP(prep);
  auto* ctx = new (std::nothrow) ecc_context_s();
  if (!ctx) return fail(ECC_ERR_OUT_OF_MEMORY, "context allocation failed");
  ctx->device = hip_device;
  *out = ctx;
  return ECC_OK;
}

ecc_status ecc_destroy(ecc_context ctx) {
  if (!ctx) return ECC_OK;
  DeviceGuard dg(ctx->device);
  (void)hipDeviceSynchronize();
  for (ecc_filter_plan p : ctx->plans) delete p;   // plans still alive go with the context
  ctx->plans.clear();
  destroy_volume_plans(ctx);
  if (ctx->ws_event) (void)hipEventDestroy(ctx->ws_event);
  delete ctx;
  return ECC_OK;
}

ecc_status ecc_fft_size(ecc_context ctx, int n, int R, int* P) {
  ECC_REQ(ctx && P, "NULL argument");
  ECC_REQ(n >= 1 && R >= 0 && n + R <= 16384, "size out of range");
  *P = fft_size_for(ctx, n, R);
  return ECC_OK;
}

ecc_status ecc_set_stage_events(ecc_context ctx, void* const* events, int n) {
  ECC_REQ(ctx, "NULL context");
  ECC_REQ(n >= 0 && n <= 64, "n must be in [0, 64]");
  ctx->stage_events.clear();
  if (events && n > 0)
    for (int i = 0; i < n; ++i) ctx->stage_events.push_back(static_cast<hipEvent_t>(events[i]));
  return ECC_OK;
}

ecc_status ecc_set_autotune(ecc_context ctx, int enable) {
  ECC_REQ(ctx, "NULL context");
  ctx->autotune = enable ? 1 : 0;
  return ECC_OK;
}

ecc_status ecc_set_strategy(ecc_context ctx, ecc_strategy strategy) {
  ECC_REQ(ctx, "NULL context");
  ECC_REQ(strategy == ECC_STRATEGY_AUTO || strategy == ECC_STRATEGY_TWO_PASS || strategy == ECC_STRATEGY_TILED ||
              strategy == ECC_STRATEGY_DIRECT,
          "unknown strategy");
  ctx->strategy = strategy;
  return ECC_OK;
}

ecc_status ecc_filter_plan_create(ecc_context ctx, ecc_group group, const float* filter, int Sz,
                                  int K, const ecc_group_params* gp, void* stream,
                                  ecc_filter_plan* out) {
  ECC_REQ(ctx && out, "NULL argument");
  *out = nullptr;
  DeviceGuard dg(ctx->device);
  hipStream_t st = S(stream);
  auto plan = std::make_unique<ecc_filter_plan_s>();
  plan->ctx = ctx;
  plan->device = ctx->device;
  plan->group = group;
  if (group == ECC_GROUP_ROTATION) {
    ECC_REQ(filter != nullptr, "filter is NULL");
    ECC_REQ(Sz >= 3 && Sz <= 255 && Sz % 2 == 1, "S must be odd, 3 <= S <= 255");
    const int R = (Sz - 1) / 2;
    int M = (gp && gp->angular_samples > 0) ? gp->angular_samples : 0;
    if (M == 0) {
      const int need = std::max(8 * (2 * K + 1), 4 * (int)std::ceil(2.0 * 3.14159265358979323846 * R));
      M = 1;
      while (M < need) M *= 2;
    }
    ECC_REQ(K >= 0 && 2 * K + 2 <= M, "need 0 <= K <= M/2 - 1");
    ECC_REQ(M <= 2048, "angular_samples must be <= 2048");
    plan->S = Sz;
    plan->R = R;
    plan->K = K;
    plan->U = K + 1;
    plan->M = M;
    // distinct squared radii and the radius index of every window pixel
    std::vector<int> d2list;
    for (int d2 = 1; d2 <= R * R; ++d2) {
      bool hit = false;
      for (int a = 0; a <= R && !hit; ++a) {
        const int b2 = d2 - a * a;
        if (b2 < 0) break;
        const int b = (int)std::lround(std::sqrt((double)b2));
        if (b * b == b2) hit = true;
      }
      if (hit) d2list.push_back(d2);
    }
    std::vector<int> rmap(Sz * Sz, -1);
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const int d2 = dx * dx + dy * dy;
        if (d2 == 0 || d2 > R * R) continue;
        rmap[(dy + R) * Sz + (dx + R)] =
            (int)(std::lower_bound(d2list.begin(), d2list.end(), d2) - d2list.begin());
      }
    const int nrad = (int)d2list.size();
    DevBuf dd2, drmap, fk;
    ECC_HIP(dd2.ensure(std::max(1, nrad) * sizeof(int)));
    ECC_HIP(drmap.ensure(rmap.size() * sizeof(int)));
    ECC_HIP(fk.ensure((size_t)std::max(1, nrad) * plan->U * sizeof(cx<double>)));
    ECC_HIP(plan->comps64.ensure((size_t)plan->U * Sz * Sz * sizeof(cx<double>)));
    if (nrad) ECC_HIP(hipMemcpyAsync(dd2.p, d2list.data(), nrad * sizeof(int), hipMemcpyHostToDevice, st));
    ECC_HIP(hipMemcpyAsync(drmap.p, rmap.data(), rmap.size() * sizeof(int), hipMemcpyHostToDevice, st));
    if (nrad) ECC_HIP(launch_polar_dft(st, filter, Sz, K, M, dd2.as<int>(), nrad, fk.as<cx<double>>()));
    ECC_HIP(launch_synth_rotation(st, filter, Sz, K, drmap.as<int>(), fk.as<cx<double>>(),
                                  plan->comps64.as<cx<double>>()));
    plan->weights.assign(plan->U, 2.f);
    plan->weights[0] = 1.f;
    plan->parity.resize(plan->U);
    for (int k = 0; k < plan->U; ++k) plan->parity[k] = (k % 2) ? -1.f : 1.f;
    plan->symmetric = 1;
    ECC_HIP(hipStreamSynchronize(st));   // temporaries above are freed on return
  } else if (group == ECC_GROUP_SCALE) {
    ECC_REQ(filter == nullptr, "scale plans build their Gaussian from gp; filter must be NULL");
    ScaleSetup s{};
    ECC_TRY(scale_setup(gp, s));
    scale_plan_fields(plan.get(), s);
    ECC_HIP(plan->comps64.ensure((size_t)plan->U * plan->S * plan->S * sizeof(cx<double>)));
    ECC_HIP(launch_scale_components(st, s.sigma0, s.u_lo, s.u_hi, s.L, s.n, s.R,
                                    plan->comps64.as<cx<double>>()));
    plan->parity.assign(plan->U, 1.f);   // radial components: F_k(-x) = F_k(x)
    plan->symmetric = 1;
  } else if (group == ECC_GROUP_ROTATION_SCALE) {
    ECC_REQ(filter != nullptr, "filter is NULL");
    ECC_REQ(Sz >= 3 && Sz <= 255 && Sz % 2 == 1, "S must be odd, 3 <= S <= 255");
    const int R = (Sz - 1) / 2;
    const int n = (gp && gp->scale_components > 0) ? gp->scale_components : 9;
    const double smin = (gp && gp->scale_min > 0) ? gp->scale_min : 1.0;
    const double smax = (gp && gp->scale_max > 0) ? gp->scale_max : 2.0;
    const double fac = (gp && gp->scale_period_factor > 0) ? gp->scale_period_factor : 1.5;
    ECC_REQ(n % 2 == 1 && n <= 255, "scale_components must be odd and <= 255 for joint plans");
    ECC_REQ(smin <= smax && fac >= 1.0, "need scale_min <= scale_max and scale_period_factor >= 1");
    int M = (gp && gp->angular_samples > 0) ? gp->angular_samples : 0;
    if (M == 0) {
      const int need = std::max(8 * (2 * K + 1), 4 * (int)std::ceil(2.0 * 3.14159265358979323846 * R));
      M = 1;
      while (M < need) M *= 2;
    }
    ECC_REQ(K >= 0 && 2 * K + 2 <= M && M <= 2048, "need 0 <= K <= M/2 - 1 and angular_samples <= 2048");
    const double u_lo = -std::log(smax), u_hi = std::log((double)R) - std::log(smin);
    const double L = fac * (u_hi - u_lo);
    ECC_REQ(L > 0.0, "empty log-radial range (R = 1 with scale_min = scale_max = 1)");
    const int U = (K + 1) * n - (n - 1) / 2;
    ECC_REQ(U <= 4096, "too many components");
    plan->S = Sz;
    plan->R = R;
    plan->K = K;
    plan->U = U;
    plan->M = M;
    plan->joint_n = n;
    plan->joint_om1 = 2.0 * 3.14159265358979323846 / L;
    DevBuf ftmp, ctmp;
    ECC_HIP(ftmp.ensure((size_t)(n + 2) * (2 * K + 1) * sizeof(cx<double>)));
    ECC_HIP(ctmp.ensure((size_t)(2 * K + 1) * n * sizeof(cx<double>)));
    ECC_HIP(plan->comps64.ensure((size_t)U * Sz * Sz * sizeof(cx<double>)));
    ECC_HIP(launch_joint_components(st, filter, Sz, K, M, n, u_lo, u_hi, L, ftmp.as<cx<double>>(),
                                    ctmp.as<cx<double>>(), plan->comps64.as<cx<double>>()));
    plan->weights.assign(U, 2.f);
    plan->weights[0] = 1.f;
    plan->parity.resize(U);
    {
      const int h = (n - 1) / 2;
      for (int c = 0; c < U; ++c) {
        const int k = c <= h ? 0 : 1 + (c - (h + 1)) / n;
        plan->parity[c] = (k % 2) ? -1.f : 1.f;   // F_{k,l}(-x) = (-1)^k F_{k,l}(x)
      }
    }
    plan->symmetric = 1;
    ECC_HIP(hipStreamSynchronize(st));   // temporaries above are freed on return
  } else {
    return fail(ECC_ERR_INVALID_ARGUMENT, "unknown group");
  }
  ECC_TRY(finish_plan(plan.get(), st));
  *out = plan.release();
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->plans.insert(*out);
  return ECC_OK;
}

ecc_status ecc_filter_plan_from_components(ecc_context ctx, ecc_group group, const float* comps,
                                           int Sz, int K, const ecc_group_params* gp,
                                           void* stream, ecc_filter_plan* out) {
  ECC_REQ(ctx && out && comps, "NULL argument");
  *out = nullptr;
  ECC_REQ(Sz >= 1 && Sz <= 255 && Sz % 2 == 1, "S must be odd, 1 <= S <= 255");
  ECC_REQ(K >= 0 && K <= 255, "K out of range");
  ECC_REQ(((uintptr_t)comps & 7) == 0, "components must be 8-byte aligned");
  DeviceGuard dg(ctx->device);
  hipStream_t st = S(stream);
  auto plan = std::make_unique<ecc_filter_plan_s>();
  plan->ctx = ctx;
  plan->device = ctx->device;
  plan->group = group;
  if (group == ECC_GROUP_SCALE) {
    ScaleSetup s{};
    ECC_TRY(scale_setup(gp, s));
    scale_plan_fields(plan.get(), s);
    ECC_REQ(K + 1 == plan->U, "scale plans need K + 1 = scale_components / 2 + 1 components");
  } else if (group == ECC_GROUP_ROTATION) {
    plan->weights.assign(K + 1, 2.f);
    plan->weights[0] = 1.f;
  } else {
    return fail(ECC_ERR_INVALID_ARGUMENT, "unknown group (rotation-and-scale plans are built from a filter only)");
  }
  plan->S = Sz;
  plan->R = (Sz - 1) / 2;
  plan->K = K;
  plan->U = K + 1;
  plan->M = 0;
  plan->symmetric = 0;   // arbitrary components: keep full-plane spectra
  const size_t n = (size_t)plan->U * Sz * Sz;
  ECC_HIP(plan->comps64.ensure(n * sizeof(cx<double>)));
  ECC_HIP(launch_f2d(st, reinterpret_cast<const cx<float>*>(comps), plan->comps64.as<cx<double>>(), (long long)n));
  ECC_TRY(finish_plan(plan.get(), st));
  *out = plan.release();
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->plans.insert(*out);
  return ECC_OK;
}

ecc_status ecc_filter_plan_get_components(ecc_filter_plan plan, float* out, void* stream) {
  ECC_REQ(plan && out, "NULL argument");
  DeviceGuard dg(plan->ctx->device);
  ECC_HIP(hipMemcpyAsync(out, plan->comps32.p, (size_t)plan->U * plan->S * plan->S * sizeof(cx<float>),
                         hipMemcpyDeviceToDevice, S(stream)));
  return ECC_OK;
}

ecc_status ecc_filter_plan_info(ecc_filter_plan plan, int* Sz, int* K, int* M) {
  ECC_REQ(plan, "NULL plan");
  if (Sz) *Sz = plan->S;
  if (K) *K = plan->K;
  if (M) *M = plan->M;
  return ECC_OK;
}

ecc_status ecc_filter_plan_component_count(ecc_filter_plan plan, int* U) {
  ECC_REQ(plan && U, "NULL argument");
  *U = plan->U;
  return ECC_OK;
}

ecc_status ecc_filter_plan_destroy(ecc_filter_plan plan) {
  if (!plan) return ECC_OK;
  DeviceGuard dg(plan->device);
  (void)hipDeviceSynchronize();
  {
    std::lock_guard<std::mutex> g(plan->ctx->mu);
    plan->ctx->plans.erase(plan);
  }
  delete plan;
  return ECC_OK;
}

}  // extern "C"

// =====================================================================================
namespace {

struct Geometry {
  int ny, nx, Py, Px, W;
  const Transform *Tx, *Ty;
  const Spectrum* sp;
};

ecc_status geometry(ecc_context ctx, ecc_filter_plan plan, int ny, int nx, hipStream_t st, Geometry& g) {
  g.ny = ny;
  g.nx = nx;
  g.Py = fft_size_for(ctx, ny, plan->R);
  g.Px = fft_size_for(ctx, nx, plan->R);
  g.W = g.Px / 2 + 1;
  ECC_HIP(get_transform(ctx, g.Py, &g.Ty));
  ECC_HIP(get_transform(ctx, g.Px, &g.Tx));
  ECC_TRY(get_spectrum(plan, g.Py, g.Px, st, &g.sp));
  return ECC_OK;
}

}  // namespace
namespace ecc {
ecc_status validate_images(ecc_filter_plan plan, int batch, int ny, int nx, bool joint) {
  ECC_REQ(joint == (plan->group == ECC_GROUP_ROTATION_SCALE),
          joint ? "ecc_joint_convolution needs a rotation-and-scale plan"
                : "rotation-and-scale plans need both fields: use ecc_joint_convolution");
  ECC_REQ(batch >= 1 && batch <= 65535, "batch must be in [1, 65535]");
  ECC_REQ(ny >= 1 && nx >= 1 && ny <= 4096 && nx <= 4096, "image sides must be in [1, 4096]");
  ECC_REQ(plan->S <= std::min(ny, nx) || plan->group == ECC_GROUP_SCALE,
          "filter window larger than the image");
  return ECC_OK;
}
}  // namespace ecc
namespace {


// Correlation-type stack: T_k = IFFT_y(Hh . filter product) for k = 0..U-1.
// Forward transform of the signal (once) and the component stack for components
// [kb, kb + kn): T_k = IFFT_y(Hh . filter product). With fwd = false the signal spectrum
// of the previous call is reused (same signal, next chunk of components).
ecc_status corr_stack(ecc_context ctx, ecc_filter_plan plan, const Geometry& g, int batch,
                      const float* H, long long planeH, int ldH, int conj_mode, hipStream_t st,
                      cx<float>** T_out, long long* planeTk, long long* planeTimg, int kb = 0,
                      int kn = -1, bool fwd = true) {
  const int ny = g.ny, nx = g.nx, Py = g.Py, Px = g.Px, W = g.W;
  if (kn < 0) kn = plan->U - kb;
  const int U = kn;
  const int ldW = pitch16(W);
  const long long pA = (long long)ny * ldW, pH = (long long)Py * ldW, pTk = 2LL * ny * ldW,
                  pTi = pTk * U;
  const size_t need = ws_corr_stack(batch, ny, Py, Px, U);
  if (fwd) ECC_HIP(ctx->ws.ensure(need));
  else if (ctx->ws.n < need) return fail(ECC_ERR_INTERNAL, "component chunk larger than the first");
  cx<float>* A = ctx->ws.as<cx<float>>();
  cx<float>* Hh = A + batch * pA;
  cx<float>* T = Hh + batch * pH;
  RowCfg r1 = row_config(*g.Tx, Px, sizeof(cx<float>));
  ColCfg c2 = col_config(*g.Ty, 2, sizeof(cx<float>), 512);
  ColCfg c3 = corr_col_config(*g.Ty);
  ECC_TRY(check_cfg_row(r1, *g.Tx, sizeof(cx<float>), "row"));
  ECC_TRY(check_cfg_col(c2, *g.Ty, sizeof(cx<float>), "column", false));
  ECC_TRY(check_cfg_col(c3, *g.Ty, sizeof(cx<float>), "column", true));
  if (fwd) {
    mark(ctx, 0, st);
    ECC_HIP(launch_rows_r2c(st, r1, batch, H, planeH, ldH, A, pA, ldW, ny, nx, W, g.Tx->desc, g.Tx->f()));
    mark(ctx, 1, st);
    ECC_HIP(launch_cols_fwd(st, c2, batch, A, pA, ldW, ny, W, Hh, pH, ldW, g.Ty->desc, g.Ty->f()));
    mark(ctx, 2, st);
  }
  const cx<float>* Fspec = g.sp->buf.as<cx<float>>() + (long long)kb * Py * g.sp->ld;
  const int nblk = (W + (1 << c3.lgB) - 1) >> c3.lgB;
  // components per workgroup: enough workgroups for about 2048 in flight
  const int kchunk = std::min(U, std::max(1, (U * nblk * batch + 2047) / 2048));
  const float* par = plan->symmetric ? plan->d_parity.as<float>() + kb : nullptr;
  ECC_HIP(launch_corr_cols(st, c3, batch, kchunk, Hh, pH, ldW, Fspec,
                           (long long)Py * g.sp->ld, g.sp->ld, g.sp->full, par, T, pTk, pTi, ldW,
                           ny, Px, W, U, conj_mode, g.Ty->desc, g.Ty->f()));
  if (fwd) mark(ctx, 3, st);
  *T_out = T;
  *planeTk = pTk;
  *planeTimg = pTi;
  return ECC_OK;
}

// Convolution-type output: C = IFFT_y(sum_k w_k FFT_y(B_k) Fh_k) from the row stack B.
ecc_status conv_stack_rows(ecc_context ctx, ecc_filter_plan plan, const Geometry& g, int batch, const float* H,
                           long long planeH, int ldH, const Field& fld, int sig_norm, int nsig,
                           cx<float>* Bk, hipStream_t st) {
  const int ny = g.ny, nx = g.nx, Px = g.Px, U = plan->U;
  const long long pBk = (long long)ny * Px, pBs = pBk * U, pBi = pBs * nsig;
  RowCfg r1 = row_config(*g.Tx, nx, sizeof(cx<float>));
  ECC_TRY(check_cfg_row(r1, *g.Tx, sizeof(cx<float>), "row"));
  mark(ctx, 0, st);
  ECC_HIP(launch_conv_rows_fwd(st, r1, batch, H, planeH, ldH, fld, sig_norm, nsig, Bk, pBk, pBs, pBi,
                               Px, ny, nx, U, g.Tx->desc, g.Tx->f()));
  mark(ctx, 1, st);
  return ECC_OK;
}

ecc_status conv_finish(ecc_context ctx, ecc_filter_plan plan, const Geometry& g, int batch, const cx<float>* Bk, int nsig,
                       cx<float>* C, float* y, long long planeY, int ldY, hipStream_t st) {
  const int ny = g.ny, nx = g.nx, Py = g.Py, Px = g.Px, U = plan->U;
  const long long pBk = (long long)ny * Px, pBs = pBk * U, pBi = pBs * nsig;
  const long long pCs = (long long)ny * Px, pCi = pCs * nsig;
  ColCfg c2 = col_config(*g.Ty, 2, sizeof(cx<float>), 512);
  RowCfg r3 = row_config(*g.Tx, nx, sizeof(cx<float>));
  ECC_TRY(check_cfg_col(c2, *g.Ty, sizeof(cx<float>), "column", true));
  ECC_TRY(check_cfg_row(r3, *g.Tx, sizeof(cx<float>), "row"));
  const float* par = plan->symmetric ? plan->d_parity.as<float>() : nullptr;
  // the partial planes of the component groups follow C in the workspace
  const int G = conv_col_groups(batch, Px, U);
  cx<float>* part = C + (long long)batch * nsig * ny * Px;
  ECC_HIP(launch_conv_cols(st, c2, batch, Bk, pBk, pBs, pBi, Px, g.sp->buf.as<cx<float>>(),
                           (long long)Py * g.sp->ld, g.sp->ld, g.sp->full, par,
                           plan->d_weights.as<float>(), C, pCs, pCi, Px, ny, Py, Px, g.W, U, nsig,
                           g.Ty->desc, g.Ty->f(), G, part));
  mark(ctx, 2, st);
  ECC_HIP(launch_conv_rows_inv(st, r3, batch, C, pCs, pCi, Px, y, planeY, ldY, ny, nx, nsig,
                               1.0f / ((float)Py * (float)Px), g.Tx->desc, g.Tx->f()));
  mark(ctx, 3, st);
  return ECC_OK;
}

// Row transforms + per-pixel combination of a correlation-type stack.
ecc_status corr_rows(ecc_filter_plan plan, const Geometry& g, int batch, const cx<float>* T, long long pTk,
                     long long pTi, const Field& fl, float* y, long long planeY, int ldY, float scl,
                     float* y2, const float* mulsig, long long planeMul, int ldMul, hipStream_t st,
                     int kb = 0, int kn = -1, int accum = 0) {
  if (kn < 0) kn = plan->U - kb;
  const int U = kn;
  const float* wts = plan->d_weights.as<float>() + kb;
  if (g.Tx->fR0 > 0) {
    const int NR = 4;   // image rows per workgroup
    ECC_HIP(launch_corr_rows_fixed(st, NR, batch, T, pTk, pTi, pitch16(g.W), fl, y, planeY, ldY, g.ny, g.nx, U,
                                   wts, scl, y2, mulsig, planeMul, ldMul, 1.0f, kb, accum, g.Px,
                                   g.Tx->fx()));
    return ECC_OK;
  }
  RowCfg r4 = row_config(*g.Tx, g.nx, sizeof(cx<float>));
  // two component transforms of up to 256 threads per workgroup: rows that need 512
  // threads (above 4096 points, or more than 1024 butterflies per pass) are refused
  if (r4.TF > 256)
    return fail(ECC_ERR_UNSUPPORTED, "row transform too long for the two-pass correlation's row kernel");
  r4.B = 2;
  ECC_TRY(check_cfg_row(r4, *g.Tx, sizeof(cx<float>), "row"));
  ECC_HIP(launch_corr_rows(st, r4, batch, T, pTk, pTi, pitch16(g.W), fl, y, planeY, ldY, g.ny, g.nx, U,
                           wts, scl, y2, mulsig, planeMul, ldMul, 1.0f, kb, accum, g.Tx->desc,
                           g.Tx->f()));
  return ECC_OK;
}

}  // namespace
namespace ecc {
Field make_field(ecc_filter_plan plan, const float* f, long long plane, int ld, double mul_sign) {
  Field fl;
  fl.ptr = f;
  fl.plane = plane;
  fl.ld = ld;
  fl.log_mode = plan->log_mode;
  fl.mul = plan->field_mul * mul_sign;
  fl.add = 0.0;
  return fl;
}
}  // namespace ecc
namespace {


// Strategy of a forward call: TILED needs a block shape; AUTO takes the tiled path when
// a block shape with side >= the filter diameter exists (the halo then costs at most ~4x
// the block in transform work); everything else runs TWO_PASS. With allow_direct (the
// forward correlation and convolution of ecc_extended), DIRECT runs the spatial sums when
// the filter side has a kernel, and AUTO takes them when direct_preferred says they are
// faster than the block path. Calls without allow_direct treat DIRECT as AUTO.
ecc_status resolve_strategy(ecc_context ctx, ecc_op op, ecc_filter_plan plan, int ny, int nx, int batch,
                            ecc_strategy* used, TileChoice* tc, bool allow_direct = false) {
  *used = ECC_STRATEGY_TWO_PASS;
  const bool direct_ok = allow_direct && direct_supported(plan->S);
  if (ctx->strategy == ECC_STRATEGY_DIRECT && allow_direct) {
    if (!direct_ok) return fail(ECC_ERR_UNSUPPORTED, "the direct kernels take filter sides 3..15");
    *used = ECC_STRATEGY_DIRECT;
    return ECC_OK;
  }
  const ecc_strategy want = ctx->strategy == ECC_STRATEGY_DIRECT ? ECC_STRATEGY_AUTO : ctx->strategy;
  auto pick = [&](int min_T) {
    return op == ECC_CORRELATION ? pick_tile(ctx, plan->R, plan->U, ny, nx, batch, false, min_T, *tc)
                                 : pick_tile_conv(ctx, plan->R, plan->U, ny, nx, batch, min_T, *tc);
  };
  if (want == ECC_STRATEGY_TILED) {
    if (!pick(16)) return fail(ECC_ERR_UNSUPPORTED, "no block shape for this filter radius (tiled strategy)");
    *used = ECC_STRATEGY_TILED;
  } else if (want == ECC_STRATEGY_AUTO && pick(2 * plan->R)) {
    *used = ECC_STRATEGY_TILED;
  }
  if (want == ECC_STRATEGY_AUTO && direct_ok &&
      direct_preferred(ctx, op == ECC_CONVOLUTION, plan->S, plan->U, ny, nx, batch))
    *used = ECC_STRATEGY_DIRECT;
  return ECC_OK;
}

}  // namespace
namespace ecc {
ecc_status forward_impl(ecc_context ctx, ecc_op op, ecc_filter_plan plan, int batch, int ny, int nx,
                        const float* signal, int ld_signal, const float* field, int ld_field,
                        float* out, int ld_out, hipStream_t st, void* saved) {
  const long long pS = (long long)ny * ld_signal, pF = (long long)ny * ld_field, pO = (long long)ny * ld_out;
  if (ctx->autotune) ECC_TRY(calibrate_tiles(ctx, st));
  ecc_strategy strat;
  TileChoice tc;
  ECC_TRY(resolve_strategy(ctx, op, plan, ny, nx, batch, &strat, &tc, saved == nullptr));
  if (saved) strat = ECC_STRATEGY_TWO_PASS;   // the saved stack is the two-pass form's row stack
  if (strat == ECC_STRATEGY_DIRECT) {
    TileArgs a{};
    a.H = signal;
    a.planeH = pS;
    a.ldH = ld_signal;
    a.fld = make_field(plan, field, pF, ld_field, 1.0);
    a.y = out;
    a.planeY = pO;
    a.ldY = ld_out;
    a.ny = ny;
    a.nx = nx;
    a.R = plan->R;
    a.U = plan->U;
    a.kofs = 0;
    a.w = plan->d_weights.as<float>();
    a.scale = 1.0f;
    a.Fs = plan->comps32.as<cx<float>>();
    mark(ctx, 0, st);
    ECC_HIP(launch_direct(st, op == ECC_CONVOLUTION, plan->S, batch, a));
    mark(ctx, 1, st);
    return ECC_OK;
  }
  TileChoice rc;
  if (strat == ECC_STRATEGY_TILED && op == ECC_CONVOLUTION && tc.N == 128 && pick_tile_ratio(plan, rc)) {
    // 128-point blocks: overlap-add (sources T x T per block, pruned forward transforms;
    // the overlap-save form holds too many registers at this size), regions added by a
    // second kernel
    const Spectrum* sp = nullptr;
    ECC_TRY(get_tile_spectrum(plan, rc.N, st, &sp, SPEC_RATIO));
    WsUse wu(ctx, st);
    ECC_HIP(ctx->ws.ensure(tratio_scratch_bytes(rc.N, rc.T, batch, ny, nx)));
    TileRatioArgs ra{};
    ra.H = signal;
    ra.planeH = pS;
    ra.ldH = ld_signal;
    ra.fld = make_field(plan, field, pF, ld_field, 1.0);
    ra.sig_norm = 0;
    ra.y = out;
    ra.planeY = pO;
    ra.ldY = ld_out;
    ra.ny = ny;
    ra.nx = nx;
    ra.R = plan->R;
    ra.T = rc.T;
    ra.U = plan->U;
    ra.Fs = sp->buf.as<float2>();
    ra.par = plan->d_parity.as<float>();
    ra.part = ctx->ws.as<cx<float>>();
    mark(ctx, 0, st);
    ECC_HIP(launch_tile_ratio(st, rc.N, rc.TV, batch, ra, 0, true));
    mark(ctx, 1, st);
    return ECC_OK;
  }
  if (strat == ECC_STRATEGY_TILED && op == ECC_CONVOLUTION) {
    const Spectrum* sp = nullptr;
    ECC_TRY(get_tile_spectrum(plan, tc.N, st, &sp, SPEC_CONV));
    TileConvArgs ca{};
    ca.H = signal;
    ca.planeH = pS;
    ca.ldH = ld_signal;
    ca.fld = make_field(plan, field, pF, ld_field, 1.0);
    ca.sig_norm = 0;
    ca.nsig = 1;
    ca.y = out;
    ca.planeY = pO;
    ca.ldY = ld_out;
    ca.ny = ny;
    ca.nx = nx;
    ca.R = plan->R;
    ca.T = tc.T;
    ca.U = plan->U;
    ca.w = plan->d_weights.as<float>();
    ca.scale = 1.0f / ((float)tc.N * (float)tc.N);
    ca.Fs = sp->buf.as<cx<float>>();
    mark(ctx, 0, st);
    ECC_HIP(launch_tile_conv(st, tc.N, tc.TV, batch, ca));
    mark(ctx, 1, st);
    return ECC_OK;
  }
  if (strat == ECC_STRATEGY_TILED) {
    const Spectrum* sp = nullptr;
    const bool sym = tile_symmetric(tc.N, tc.TV) && rotation_parity(plan);
    ECC_TRY(get_tile_spectrum(plan, tc.N, st, &sp, sym ? SPEC_CENTRED : SPEC_CORR));
    Field fl = make_field(plan, field, pF, ld_field, 1.0);
    mark(ctx, 0, st);
    ECC_HIP(launch_tile_corr(st, tc.N, tc.TV, batch, signal, pS, ld_signal, fl, out, pO, ld_out, ny, nx,
                             plan->R, tc.T, plan->U, 0, plan->d_weights.as<float>(),
                             1.0f / ((float)tc.N * (float)tc.N), sp->buf.as<cx<float>>(), sym));
    mark(ctx, 1, st);
    return ECC_OK;
  }
  WsUse wu(ctx, st);
  Geometry g{};
  ECC_TRY(geometry(ctx, plan, ny, nx, st, g));
  if (op == ECC_CORRELATION) {
    const int U = plan->U;
    Field fl = make_field(plan, field, pF, ld_field, 1.0);
    cx<float>* T;
    long long pTk, pTi;
    ECC_TRY(corr_stack(ctx, plan, g, batch, signal, pS, ld_signal, 0, st, &T, &pTk, &pTi, 0, U, true));
    ECC_TRY(corr_rows(plan, g, batch, T, pTk, pTi, fl, out, pO, ld_out,
                      1.0f / ((float)g.Py * (float)g.Px), nullptr, nullptr, 0, 0, st, 0, U, 0));
    mark(ctx, 4, st);
    return ECC_OK;
  }
  const long long pB = (long long)batch * plan->U * ny * g.Px;
  ECC_HIP(ctx->ws.ensure(ws_conv_two_pass(batch, ny, g.Py, g.Px, plan->U, 1, saved != nullptr)));
  cx<float>* Bk = saved ? static_cast<cx<float>*>(saved) : ctx->ws.as<cx<float>>();
  cx<float>* C = saved ? ctx->ws.as<cx<float>>() : ctx->ws.as<cx<float>>() + pB;
  Field fl = make_field(plan, field, pF, ld_field, 1.0);
  ECC_TRY(conv_stack_rows(ctx, plan, g, batch, signal, pS, ld_signal, fl, 0, 1, Bk, st));
  ECC_TRY(conv_finish(ctx, plan, g, batch, Bk, 1, C, out, pO, ld_out, st));
  return ECC_OK;
}
}  // namespace ecc
namespace {


}  // namespace

extern "C" {

ecc_status ecc_extended(ecc_context ctx, ecc_op op, ecc_filter_plan plan, int batch, int ny, int nx,
                        const float* signal, int ld_signal, const float* field, int ld_field,
                        float* out, int ld_out, ecc_precision prec, void* stream) {
  ECC_REQ(ctx && plan, "NULL context or plan");
  ECC_REQ(plan->ctx == ctx, "plan belongs to another context");
  ECC_REQ(signal && field && out, "NULL image pointer");
  ECC_REQ(op == ECC_CORRELATION || op == ECC_CONVOLUTION, "unknown op");
  if (prec != ECC_PREC_FP32)
    return fail(ECC_ERR_UNSUPPORTED, "only ECC_PREC_FP32 is implemented for ecc_extended");
  ECC_TRY(validate_images(plan, batch, ny, nx));
  ECC_REQ(ld_signal >= nx && ld_field >= nx && ld_out >= nx, "row strides must be >= nx");
  const size_t bo = (size_t)batch * ny * ld_out * sizeof(float);
  ECC_REQ(!overlaps(out, bo, signal, (size_t)batch * ny * ld_signal * sizeof(float)) &&
              !overlaps(out, bo, field, (size_t)batch * ny * ld_field * sizeof(float)),
          "out aliases an input");
  DeviceGuard dg(ctx->device);
  return forward_impl(ctx, op, plan, batch, ny, nx, signal, ld_signal, field, ld_field, out, ld_out,
                      S(stream), nullptr);
}

ecc_status ecc_describe(ecc_context ctx, ecc_op op, ecc_filter_plan plan, int ny, int nx,
                        ecc_strategy* strategy, int* fft_size, int* block) {
  ECC_REQ(ctx && plan, "NULL context or plan");
  ECC_REQ(op == ECC_CORRELATION || op == ECC_CONVOLUTION, "unknown op");
  const bool joint = plan->group == ECC_GROUP_ROTATION_SCALE;
  ECC_REQ(!joint || op == ECC_CONVOLUTION, "rotation-and-scale plans have the convolution only");
  ECC_TRY(validate_images(plan, 1, ny, nx, joint));
  ecc_strategy used;
  TileChoice tc;
  if (ctx->autotune) {
    DeviceGuard dg(ctx->device);
    ECC_TRY(calibrate_tiles(ctx, nullptr));
  }
  ECC_TRY(resolve_strategy(ctx, op, plan, ny, nx, 1, &used, &tc, true));
  if (strategy) *strategy = used;
  if (fft_size)
    *fft_size = used == ECC_STRATEGY_TILED ? tc.N : used == ECC_STRATEGY_DIRECT ? 0 : fft_size_for(ctx, ny, plan->R);
  if (block) *block = used == ECC_STRATEGY_TILED ? tc.T : 0;
  return ECC_OK;
}

ecc_status ecc_scale_smooth(ecc_context ctx, ecc_filter_plan plan, int ny, int nx, const float* signal,
                            int ld_signal, const float* scale_, int ld_scale, float* out, int ld_out,
                            ecc_precision prec, void* stream) {
  ECC_REQ(ctx && plan, "NULL context or plan");
  ECC_REQ(plan->group == ECC_GROUP_SCALE, "ecc_scale_smooth needs a scale plan");
  return ecc_normalized_convolution(ctx, plan, 1, ny, nx, signal, ld_signal, scale_, ld_scale, out, ld_out, prec,
                                    stream);
}

ecc_status ecc_normalized_convolution(ecc_context ctx, ecc_filter_plan plan, int batch, int ny, int nx,
                                      const float* signal, int ld_signal, const float* field, int ld_field,
                                      float* out, int ld_out, ecc_precision prec, void* stream) {
  ECC_REQ(ctx && plan, "NULL context or plan");
  ECC_REQ(plan->ctx == ctx, "plan belongs to another context");
  ECC_REQ(signal && field && out, "NULL image pointer");
  ECC_REQ(prec == ECC_PREC_FP32 || prec == ECC_PREC_MFMA_FP16_HILO || prec == ECC_PREC_MFMA_BF16_HILO,
          "unknown precision");
  ECC_TRY(validate_images(plan, batch, ny, nx));
  ECC_REQ(ld_signal >= nx && ld_field >= nx && ld_out >= nx, "row strides must be >= nx");
  const size_t bo = (size_t)batch * ny * ld_out * sizeof(float);
  ECC_REQ(!overlaps(out, bo, signal, (size_t)batch * ny * ld_signal * sizeof(float)) &&
              !overlaps(out, bo, field, (size_t)batch * ny * ld_field * sizeof(float)),
          "out aliases an input");
  DeviceGuard dg(ctx->device);
  hipStream_t st = S(stream);
  const long long pS = (long long)ny * ld_signal, pF = (long long)ny * ld_field, pO = (long long)ny * ld_out;
  // the scale group divides the signal by |T(q)|^2 = s(q)^2 (eq. normalization with the
  // normalised signal); rotations keep the filter's integral and leave it as it is
  const int sig_norm = plan->sig_norm;
  if (ctx->autotune) ECC_TRY(calibrate_tiles(ctx, st));
  ecc_strategy strat;
  TileChoice tc;
  ECC_TRY(resolve_strategy(ctx, ECC_CONVOLUTION, plan, ny, nx, batch, &strat, &tc));
  TileChoice rc;
  if (strat == ECC_STRATEGY_TILED && tc.N == 128 && pick_tile_ratio(plan, rc)) {
    // overlap-add blocks: both signals in one launch, regions added by a second kernel
    const Spectrum* sp = nullptr;
    ECC_TRY(get_tile_spectrum(plan, rc.N, st, &sp, SPEC_RATIO));
    WsUse wu(ctx, st);
    ECC_HIP(ctx->ws.ensure(tratio_scratch_bytes(rc.N, rc.T, batch, ny, nx)));
    TileRatioArgs ra{};
    ra.H = signal;
    ra.planeH = pS;
    ra.ldH = ld_signal;
    ra.fld = make_field(plan, field, pF, ld_field, 1.0);
    ra.sig_norm = sig_norm;
    ra.y = out;
    ra.planeY = pO;
    ra.ldY = ld_out;
    ra.ny = ny;
    ra.nx = nx;
    ra.R = plan->R;
    ra.T = rc.T;
    ra.U = plan->U;
    ra.Fs = sp->buf.as<float2>();
    ra.par = plan->d_parity.as<float>();
    ra.part = ctx->ws.as<cx<float>>();
    mark(ctx, 0, st);
    ECC_HIP(launch_tile_ratio(st, rc.N, rc.TV, batch, ra,
                              prec == ECC_PREC_FP32 ? 0 : (prec == ECC_PREC_MFMA_FP16_HILO ? 1 : 2)));
    mark(ctx, 1, st);
    return ECC_OK;
  }
  if (prec != ECC_PREC_FP32)
    return fail(ECC_ERR_UNSUPPORTED,
                "the matrix-core precisions run in the overlap-add block kernel only (128-point blocks: filter "
                "radius above 24 under the default strategy, components with parity)");
  if (strat == ECC_STRATEGY_TILED) {
    const Spectrum* sp = nullptr;
    ECC_TRY(get_tile_spectrum(plan, tc.N, st, &sp, SPEC_CONV));
    TileConvArgs ca{};
    ca.H = signal;
    ca.planeH = pS;
    ca.ldH = ld_signal;
    ca.fld = make_field(plan, field, pF, ld_field, 1.0);
    ca.sig_norm = sig_norm;
    ca.nsig = 2;
    ca.y = out;
    ca.planeY = pO;
    ca.ldY = ld_out;
    ca.ny = ny;
    ca.nx = nx;
    ca.R = plan->R;
    ca.T = tc.T;
    ca.U = plan->U;
    ca.w = plan->d_weights.as<float>();
    ca.scale = 1.0f;
    ca.Fs = sp->buf.as<cx<float>>();
    mark(ctx, 0, st);
    ECC_HIP(launch_tile_conv(st, tc.N, tc.TV, batch, ca));
    mark(ctx, 1, st);
    return ECC_OK;
  }
  WsUse wu(ctx, st);
  Geometry g{};
  ECC_TRY(geometry(ctx, plan, ny, nx, st, g));
  const long long pB = (long long)batch * 2 * plan->U * ny * g.Px;
  ECC_HIP(ctx->ws.ensure(ws_conv_two_pass(batch, ny, g.Py, g.Px, plan->U, 2, false)));
  cx<float>* Bk = ctx->ws.as<cx<float>>();
  cx<float>* C = Bk + pB;
  Field fl = make_field(plan, field, pF, ld_field, 1.0);
  ECC_TRY(conv_stack_rows(ctx, plan, g, batch, signal, pS, ld_signal, fl, sig_norm, 2, Bk, st));
  ECC_TRY(conv_finish(ctx, plan, g, batch, Bk, 2, C, out, pO, ld_out, st));
  return ECC_OK;
}

ecc_status ecc_joint_convolution(ecc_context ctx, ecc_filter_plan plan, int batch, int ny, int nx,
                                 const float* signal, int ld_signal, const float* angle, int ld_angle,
                                 const float* scale_, int ld_scale, float* out, int ld_out, int normalized,
                                 void* stream) {
  ECC_REQ(ctx && plan, "NULL context or plan");
  ECC_REQ(plan->ctx == ctx, "plan belongs to another context");
  ECC_REQ(signal && angle && scale_ && out, "NULL image pointer");
  ECC_TRY(validate_images(plan, batch, ny, nx, true));
  ECC_REQ(ld_signal >= nx && ld_angle >= nx && ld_scale >= nx && ld_out >= nx, "row strides must be >= nx");
  const size_t bo = (size_t)batch * ny * ld_out * sizeof(float);
  ECC_REQ(!overlaps(out, bo, signal, (size_t)batch * ny * ld_signal * sizeof(float)) &&
              !overlaps(out, bo, angle, (size_t)batch * ny * ld_angle * sizeof(float)) &&
              !overlaps(out, bo, scale_, (size_t)batch * ny * ld_scale * sizeof(float)),
          "out aliases an input");
  DeviceGuard dg(ctx->device);
  hipStream_t st = S(stream);
  const int nsig = normalized ? 2 : 1, U = plan->U;
  const long long pS = (long long)ny * ld_signal, pO = (long long)ny * ld_out;
  if (ctx->autotune) ECC_TRY(calibrate_tiles(ctx, st));
  ecc_strategy strat;
  TileChoice tc;
  ECC_TRY(resolve_strategy(ctx, ECC_CONVOLUTION, plan, ny, nx, batch, &strat, &tc));
  if (strat == ECC_STRATEGY_TILED) {
    // block convolution, components taken by scale mode (no workspace)
    const Spectrum* sp = nullptr;
    ECC_TRY(get_tile_spectrum(plan, tc.N, st, &sp, SPEC_CONV));
    TileConvArgs ca{};
    ca.H = signal;
    ca.planeH = pS;
    ca.ldH = ld_signal;
    ca.fld.ptr = angle;
    ca.fld.plane = (long long)ny * ld_angle;
    ca.fld.ld = ld_angle;
    ca.fld.log_mode = 0;
    ca.fld.mul = 1.0;
    ca.fld.add = 0.0;
    ca.sig_norm = normalized ? 1 : 0;
    ca.nsig = nsig;
    ca.y = out;
    ca.planeY = pO;
    ca.ldY = ld_out;
    ca.ny = ny;
    ca.nx = nx;
    ca.R = plan->R;
    ca.T = tc.T;
    ca.U = U;
    ca.w = plan->d_weights.as<float>();
    ca.scale = normalized ? 1.0f : 1.0f / ((float)tc.N * (float)tc.N);
    ca.Fs = sp->buf.as<cx<float>>();
    ca.joint_n = plan->joint_n;
    ca.joint_K = plan->K;
    ca.joint_om1 = (float)plan->joint_om1;
    ca.jscale = scale_;
    ca.plane_s = (long long)ny * ld_scale;
    ca.ld_s = ld_scale;
    mark(ctx, 0, st);
    ECC_HIP(launch_tile_conv(st, tc.N, tc.TV, batch, ca));
    mark(ctx, 1, st);
    return ECC_OK;
  }
  WsUse wu(ctx, st);
  Geometry g{};
  ECC_TRY(geometry(ctx, plan, ny, nx, st, g));
  ECC_HIP(ctx->ws.ensure(ws_conv_two_pass(batch, ny, g.Py, g.Px, U, nsig, false)));
  cx<float>* Bk = ctx->ws.as<cx<float>>();
  cx<float>* C = Bk + (long long)batch * nsig * U * ny * g.Px;
  JointField jf{};
  jf.theta = angle;
  jf.plane_t = (long long)ny * ld_angle;
  jf.ld_t = ld_angle;
  jf.scale = scale_;
  jf.plane_s = (long long)ny * ld_scale;
  jf.ld_s = ld_scale;
  jf.om1 = plan->joint_om1;
  const long long pBk = (long long)ny * g.Px, pBs = pBk * U, pBi = pBs * nsig;
  RowCfg r1 = row_config(*g.Tx, nx, sizeof(cx<float>));
  ECC_TRY(check_cfg_row(r1, *g.Tx, sizeof(cx<float>), "row"));
  // (the joint row kernel keeps 256 threads: its per-pixel state fills the registers)
  if (r1.B * r1.TF > 256) return fail(ECC_ERR_UNSUPPORTED, "image too wide for the two-pass joint row kernel");
  mark(ctx, 0, st);
  ECC_HIP(launch_conv_rows_fwd_joint(st, r1, batch, signal, pS, ld_signal, jf, normalized ? 1 : 0, nsig, Bk, pBk,
                                     pBs, pBi, g.Px, ny, nx, U, plan->joint_n, g.Tx->desc, g.Tx->f()));
  mark(ctx, 1, st);
  ECC_TRY(conv_finish(ctx, plan, g, batch, Bk, nsig, C, out, pO, ld_out, st));
  return ECC_OK;
}

ecc_status ecc_match_rotations(ecc_context ctx, ecc_filter_plan plan, int ny, int nx, const float* signal,
                               int ld, int n_angles, float* best_score, int* best_index, int ld_out,
                               ecc_precision prec, void* stream) {
  ECC_REQ(ctx && plan, "NULL context or plan");
  ECC_REQ(plan->ctx == ctx, "plan belongs to another context");
  ECC_REQ(plan->group == ECC_GROUP_ROTATION, "matching needs a rotation plan");
  ECC_REQ(signal && best_score && best_index, "NULL pointer");
  ECC_REQ(prec == ECC_PREC_FP32 || prec == ECC_PREC_MFMA_FP16_HILO || prec == ECC_PREC_MFMA_BF16_HILO,
          "unknown precision");
  ECC_TRY(validate_images(plan, 1, ny, nx));
  ECC_REQ(ld >= nx && ld_out >= nx, "row strides must be >= nx");
  ECC_REQ(n_angles >= 2 * plan->K + 1 && n_angles <= 64, "need 2K+1 <= n_angles <= 64");
  DeviceGuard dg(ctx->device);
  hipStream_t st = S(stream);
  if (ctx->autotune) ECC_TRY(calibrate_tiles(ctx, st));
  WsUse wu(ctx, st);
  const int R = plan->R, U = plan->U;
  TileChoice tc;
  bool tiled = false;
  if (ctx->strategy != ECC_STRATEGY_TWO_PASS)
    tiled = pick_tile(ctx, R, U, ny, nx, 1, false, ctx->strategy == ECC_STRATEGY_AUTO ? 2 * R : 16, tc);
  if (ctx->strategy == ECC_STRATEGY_TILED && !tiled)
    return fail(ECC_ERR_UNSUPPORTED, "no block shape for this filter radius (tiled strategy)");
  if (tiled) {
    // component stack G_c(p) by blocks, then the angle search (float32 or matrix cores)
    const Spectrum* sp = nullptr;
    const bool sym = tile_symmetric(tc.N, tc.TV) && rotation_parity(plan);
    ECC_TRY(get_tile_spectrum(plan, tc.N, st, &sp, sym ? SPEC_CENTRED : SPEC_CORR));
    if (plan->match_tab_A != n_angles) {
      std::vector<float> tab(64 * 64, 0.f);
      for (int m = 0; m < n_angles; ++m)
        for (int c = 0; c < U; ++c) {
          const long double a = 2.0L * 3.14159265358979323846264338327950288L * ((long long)c * m % n_angles) / n_angles;
          tab[m * 64 + 2 * c] = (float)(plan->weights[c] * cosl(a));
          tab[m * 64 + 2 * c + 1] = (float)(-plan->weights[c] * sinl(a));
        }
      ECC_HIP(plan->match_tab.ensure(tab.size() * sizeof(float)));
      ECC_HIP(hipMemcpy(plan->match_tab.p, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice));
      plan->match_tab_A = n_angles;
    }
    const long long npix = (long long)ny * nx;
    ECC_HIP(ctx->ws.ensure(ws_match_tiled(ny, nx, U)));
    mark(ctx, 0, st);
    ECC_HIP(launch_tile_stack(st, tc.N, tc.TV, signal, ld, ny, nx, R, tc.T, U, 1.0f / ((float)tc.N * (float)tc.N),
                              sp->buf.as<cx<float>>(), ctx->ws.as<float>(), sym));
    mark(ctx, 1, st);
    const int pc = prec == ECC_PREC_FP32 ? 0 : (prec == ECC_PREC_MFMA_FP16_HILO ? 1 : 2);
    ECC_HIP(launch_match_angles(st, pc, ctx->ws.as<float>(), U, npix, n_angles, plan->match_tab.as<float>(),
                                best_score, best_index, ld_out, nx));
    mark(ctx, 2, st);
    return ECC_OK;
  }
  if (prec != ECC_PREC_FP32)
    return fail(ECC_ERR_UNSUPPORTED, "the matrix-core angle search needs the tiled component stack");
  if (ctx->angle_tab_n != n_angles) {
    std::vector<float> tab(128, 0.f);
    for (int t = 0; t < n_angles; ++t) {
      const long double a = 2.0L * 3.14159265358979323846264338327950288L * t / n_angles;
      tab[t] = (float)cosl(a);
      tab[64 + t] = (float)sinl(a);
    }
    ECC_HIP(ctx->angle_tab.ensure(128 * sizeof(float)));
    ECC_HIP(hipMemcpy(ctx->angle_tab.p, tab.data(), 128 * sizeof(float), hipMemcpyHostToDevice));
    ctx->angle_tab_n = n_angles;
  }
  Geometry g{};
  ECC_TRY(geometry(ctx, plan, ny, nx, st, g));
  cx<float>* T;
  long long pTk, pTi;
  ECC_TRY(corr_stack(ctx, plan, g, 1, signal, 0, ld, 0, st, &T, &pTk, &pTi));
  // one row per workgroup, up to 512 threads, at most 2 pixels per thread (each pixel
  // keeps n_angles accumulators in registers); wider rows are split into segments of
  // 1024 pixels, each a workgroup that transforms the whole row
  RowCfg r4 = row_config(*g.Tx, nx, sizeof(cx<float>), 512);
  r4.B = 1;
  if ((nx + r4.TF - 1) / r4.TF > 2) {
    r4.TF = 512;
    const int nb = max_butterflies(*g.Tx);
    r4.NB = nb <= 512 ? 1 : (nb <= 1024 ? 2 : (nb <= 2048 ? 4 : -1));
    r4.EPX = 2;
  }
  if (r4.NB < 0 || r4.EPX < 1 || r4.EPX > 2)
    return fail(ECC_ERR_UNSUPPORTED, "transform too long for the matching kernel");
  if (lds_rows(r4, g.Tx->desc, sizeof(cx<float>)) + 64 * sizeof(cx<float>) > kMaxLds) return fail(ECC_ERR_UNSUPPORTED, "matching row transform too long");
  ECC_TRY(check_cfg_row(r4, *g.Tx, sizeof(cx<float>), "matching row"));
  ECC_HIP(launch_match_rows(st, r4, T, pTk, pitch16(g.W), best_score, best_index, ld_out, ny, nx, plan->U,
                            plan->d_weights.as<float>(), 1.0f / ((float)g.Py * (float)g.Px), n_angles,
                            ctx->angle_tab.as<float>(), g.Tx->desc, g.Tx->f()));
  mark(ctx, 4, st);
  return ECC_OK;
}

ecc_status ecc_backward_saved_size(ecc_context ctx, ecc_filter_plan plan, int batch, int ny, int nx,
                                   size_t* bytes) {
  ECC_REQ(ctx && plan && bytes, "NULL argument");
  ECC_TRY(validate_images(plan, batch, ny, nx));
  // the stack is read only by the two-pass filter gradient; with the on-chip one the
  // backward recomputes everything per block and nothing is worth saving
  if (ctx->autotune) {
    DeviceGuard dg(ctx->device);
    ECC_TRY(calibrate_tiles(ctx, nullptr));
  }
  ecc_strategy vstrat = ECC_STRATEGY_TWO_PASS;
  TileChoice vtc;
  ECC_TRY(resolve_strategy(ctx, ECC_CONVOLUTION, plan, ny, nx, batch, &vstrat, &vtc));
  if (vstrat == ECC_STRATEGY_TILED && tgradf_supported(vtc.N, vtc.TV)) {
    *bytes = 0;
    return ECC_OK;
  }
  const int Px = fft_size_for(ctx, nx, plan->R);
  *bytes = (size_t)batch * plan->U * ny * Px * sizeof(cx<float>);
  return ECC_OK;
}

ecc_status ecc_extended_save(ecc_context ctx, ecc_filter_plan plan, int batch, int ny, int nx,
                             const float* signal, const float* field, float* out, void* saved,
                             void* stream) {
  ECC_REQ(ctx && plan && signal && field && out && saved, "NULL argument");
  ECC_REQ(plan->ctx == ctx, "plan belongs to another context");
  ECC_TRY(validate_images(plan, batch, ny, nx));
  ECC_REQ(!overlaps(out, (size_t)batch * ny * nx * sizeof(float), signal, (size_t)batch * ny * nx * sizeof(float)) &&
              !overlaps(out, (size_t)batch * ny * nx * sizeof(float), field, (size_t)batch * ny * nx * sizeof(float)),
          "out aliases an input");
  DeviceGuard dg(ctx->device);
  return forward_impl(ctx, ECC_CONVOLUTION, plan, batch, ny, nx, signal, nx, field, nx, out, nx,
                      S(stream), saved);
}

// Adjoint of the extended correlation (derived from eq. Def-ECorr), with G_k = H star F_k:
//   grad_signal = Re sum_k w_k (gbar e^{-ik theta}) * F_k: the scatter of gbar e^{ik theta}
//                 with conj F_k has the same real part as its conjugate, which is the forward
//                 extended convolution of gbar;
//   grad_field  = -gbar sum_k w_k k Im(e^{ik theta} G_k): the second output of the forward
//                 correlation of H (weighted by gbar), negated;
//   grad_comps  = w_k sum_p gbar(p) e^{ik theta(p)} H(p + x): the convolution adjoint's filter
//                 part with the signal and the output gradient exchanged.
static ecc_status corr_backward(ecc_context ctx, ecc_filter_plan plan, int batch, int ny, int nx,
                                const float* signal, const float* field, const float* grad_out,
                                float* grad_signal, float* grad_comps, float* grad_field, void* stream) {
  hipStream_t st = S(stream);
  WsUse wu(ctx, st);
  const long long pI = (long long)ny * nx;
  if (grad_field) {
    DevBuf tmp;
    float* ybuf = grad_signal;   // the forward output lands here and is overwritten below
    if (!ybuf) {
      ECC_HIP(tmp.ensure((size_t)batch * pI * sizeof(float)));
      ybuf = tmp.as<float>();
    }
    ecc_strategy cstrat = ECC_STRATEGY_TWO_PASS;
    TileChoice ctc;
    ECC_TRY(resolve_strategy(ctx, ECC_CORRELATION, plan, ny, nx, batch, &cstrat, &ctc));
    Field fl = make_field(plan, field, pI, nx, 1.0);
    if (cstrat == ECC_STRATEGY_TILED && tile_has_y2(ctc.N, ctc.TV)) {
      const bool sym = tile_symmetric(ctc.N, ctc.TV) && rotation_parity(plan);
      const Spectrum* sp = nullptr;
      ECC_TRY(get_tile_spectrum(plan, ctc.N, st, &sp, sym ? SPEC_CENTRED : SPEC_CORR));
      ECC_HIP(launch_tile_corr(st, ctc.N, ctc.TV, batch, signal, pI, nx, fl, ybuf, pI, nx, ny, nx, plan->R, ctc.T,
                               plan->U, 0, plan->d_weights.as<float>(), 1.0f / ((float)ctc.N * (float)ctc.N),
                               sp->buf.as<cx<float>>(), sym, grad_field, grad_out, pI, nx));
    } else {
      Geometry g{};
      ECC_TRY(geometry(ctx, plan, ny, nx, st, g));
      cx<float>* T;
      long long pTk, pTi;
      ECC_TRY(corr_stack(ctx, plan, g, batch, signal, pI, nx, 0, st, &T, &pTk, &pTi));
      ECC_TRY(corr_rows(plan, g, batch, T, pTk, pTi, fl, ybuf, pI, nx, 1.0f / ((float)g.Py * (float)g.Px),
                        grad_field, grad_out, pI, nx, st));
    }
    ECC_HIP(launch_scale_f(st, grad_field, (long long)batch * pI, -1.0f));
    if (tmp.p) ECC_HIP(hipStreamSynchronize(st));   // tmp is freed on return
  }
  if (grad_signal)
    ECC_TRY(forward_impl(ctx, ECC_CONVOLUTION, plan, batch, ny, nx, grad_out, nx, field, nx, grad_signal, nx, st,
                         nullptr));
  if (grad_comps)
    return ecc_extended_backward(ctx, ECC_CONVOLUTION, plan, batch, ny, nx, grad_out, field, signal, nullptr,
                                 grad_comps, nullptr, nullptr, stream);
  return ECC_OK;
}

ecc_status ecc_extended_backward(ecc_context ctx, ecc_op op, ecc_filter_plan plan, int batch, int ny,
                                 int nx, const float* signal, const float* field,
                                 const float* grad_out, float* grad_signal, float* grad_comps,
                                 float* grad_field, void* saved, void* stream) {
  ECC_REQ(ctx && plan && signal && field && grad_out, "NULL argument");
  ECC_REQ(plan->ctx == ctx, "plan belongs to another context");
  ECC_REQ(op == ECC_CONVOLUTION || op == ECC_CORRELATION, "unknown op");
  ECC_REQ(plan->group == ECC_GROUP_ROTATION, "the adjoint needs a rotation plan");
  ECC_TRY(validate_images(plan, batch, ny, nx));
  DeviceGuard dg(ctx->device);
  if (op == ECC_CORRELATION) {
    ECC_REQ(!saved, "the correlation adjoint takes no saved stack");
    return corr_backward(ctx, plan, batch, ny, nx, signal, field, grad_out, grad_signal, grad_comps, grad_field,
                         stream);
  }
  hipStream_t st = S(stream);
  WsUse wu(ctx, st);
  Geometry g{};
  ECC_TRY(geometry(ctx, plan, ny, nx, st, g));
  const int Py = g.Py, Px = g.Px, W = g.W, U = plan->U, Sz = plan->S, R = plan->R;
  const long long pI = (long long)ny * nx;
  const float scl = 1.0f / ((float)Py * (float)Px);
  // grad_signal and grad_field: A_k = IFFT(Gh(w) Fh_k(-w)) combined with e^{-ik theta}
  ecc_strategy cstrat = ECC_STRATEGY_TWO_PASS;
  TileChoice ctc;
  ECC_TRY(resolve_strategy(ctx, ECC_CORRELATION, plan, ny, nx, batch, &cstrat, &ctc));
  if ((grad_signal || grad_field) && cstrat == ECC_STRATEGY_TILED && tile_has_y2(ctc.N, ctc.TV)) {
    // on chip: the tiled correlation of grad_out with F_k (spectra of conj F_k), phase
    // e^{-ik theta}, and the field part as its second output
    const bool sym = tile_symmetric(ctc.N, ctc.TV) && rotation_parity(plan);
    const Spectrum* sp = nullptr;
    ECC_TRY(get_tile_spectrum(plan, ctc.N, st, &sp, sym ? SPEC_CENTRED_CONJ : SPEC_CORR_CONJ));
    Field fl = make_field(plan, field, pI, nx, -1.0);
    DevBuf tmp;
    float* gs = grad_signal;
    if (!gs) {
      ECC_HIP(tmp.ensure((size_t)batch * pI * sizeof(float)));
      gs = tmp.as<float>();
    }
    ECC_HIP(launch_tile_corr(st, ctc.N, ctc.TV, batch, grad_out, pI, nx, fl, gs, pI, nx, ny, nx, R, ctc.T, U, 0,
                             plan->d_weights.as<float>(), 1.0f / ((float)ctc.N * (float)ctc.N),
                             sp->buf.as<cx<float>>(), sym, grad_field, grad_field ? signal : nullptr, pI, nx));
    if (tmp.p) ECC_HIP(hipStreamSynchronize(st));
  } else if (grad_signal || grad_field) {
    cx<float>* T;
    long long pTk, pTi;
    ECC_TRY(corr_stack(ctx, plan, g, batch, grad_out, pI, nx, 2, st, &T, &pTk, &pTi));
    Field fl = make_field(plan, field, pI, nx, -1.0);
    DevBuf tmp;
    float* gs = grad_signal;
    if (!gs) {
      ECC_HIP(tmp.ensure((size_t)batch * pI * sizeof(float)));
      gs = tmp.as<float>();
    }
    ECC_TRY(corr_rows(plan, g, batch, T, pTk, pTi, fl, gs, pI, nx, scl, grad_field, signal, pI, nx, st));
    if (tmp.p) ECC_HIP(hipStreamSynchronize(st));
  }
  ecc_strategy vstrat = ECC_STRATEGY_TWO_PASS;
  TileChoice vtc;
  if (grad_comps) ECC_TRY(resolve_strategy(ctx, ECC_CONVOLUTION, plan, ny, nx, batch, &vstrat, &vtc));
  if (grad_comps && vstrat == ECC_STRATEGY_TILED && tgradf_supported(vtc.N, vtc.TV)) {
    // on chip: per block and component the S x S lags of the gradient against the
    // modulated signal, then a fixed-order sum over the blocks (the saved stack, if any,
    // is not needed)
    TileGradFArgs ga{};
    ga.H = signal;
    ga.planeH = pI;
    ga.ldH = nx;
    ga.fld = make_field(plan, field, pI, nx, 1.0);
    ga.G = grad_out;
    ga.planeG = pI;
    ga.ldG = nx;
    ga.ny = ny;
    ga.nx = nx;
    ga.R = R;
    ga.T = vtc.T;
    ga.U = U;
    const long long nblk = (long long)((ny + vtc.T - 1) / vtc.T) * ((nx + vtc.T - 1) / vtc.T) * batch;
    ECC_REQ(nblk <= 0x7fffffffLL, "too many blocks");
    const size_t pbytes = ws_gradf_parts(nblk, U, Sz);
    ECC_HIP(ctx->ws.ensure(pbytes + gradf_reduce_scratch(U, Sz)));
    ga.part = ctx->ws.as<cx<float>>();
    ECC_HIP(launch_tile_gradf(st, vtc.N, vtc.TV, batch, ga));
    ECC_HIP(launch_gradf_reduce(st, ga.part, (int)nblk, U, Sz, plan->d_weights.as<float>(),
                                1.0f / ((float)vtc.N * (float)vtc.N), reinterpret_cast<cx<float>*>(grad_comps),
                                static_cast<char*>(ctx->ws.p) + pbytes));
  } else if (grad_comps) {
    // stack B_k (saved or recomputed), Gh full spectra of grad_out, D_k, small inverse
    const long long pBk = (long long)ny * Px, pBi = pBk * U;
    const long long pA = (long long)ny * W, pG = (long long)Py * W;
    const long long pD = (long long)Py * Px;
    ECC_HIP(ctx->ws.ensure(ws_gradf_two_pass(batch, ny, Py, Px, U, Sz, saved != nullptr)));
    cx<float>* A = ctx->ws.as<cx<float>>();
    cx<float>* Gh = A + batch * pA;
    cx<float>* D = Gh + batch * pG;
    cx<float>* Ts = D + U * pD;
    cx<float>* win = Ts + (long long)U * Sz * Px;
    cx<float>* Bk = saved ? static_cast<cx<float>*>(saved) : win + (long long)U * Sz * Sz;
    if (!saved) {
      Field fl = make_field(plan, field, pI, nx, 1.0);
      ECC_TRY(conv_stack_rows(ctx, plan, g, batch, signal, pI, nx, fl, 0, 1, Bk, st));
    }
    RowCfg r1 = row_config(*g.Tx, Px, sizeof(cx<float>));
    ColCfg c2 = col_config(*g.Ty, 3, sizeof(cx<float>), 512);
    ECC_TRY(check_cfg_row(r1, *g.Tx, sizeof(cx<float>), "row"));
    ECC_TRY(check_cfg_col(c2, *g.Ty, sizeof(cx<float>), "column", false));
    ECC_HIP(launch_rows_r2c(st, r1, batch, grad_out, pI, nx, A, pA, W, ny, nx, W, g.Tx->desc, g.Tx->f()));
    ECC_HIP(launch_cols_fwd(st, c2, batch, A, pA, W, ny, W, Gh, pG, W, g.Ty->desc, g.Ty->f()));
    ColCfg c3 = col_config(*g.Ty, 3, sizeof(cx<float>), 512);
    ECC_TRY(check_cfg_col(c3, *g.Ty, sizeof(cx<float>), "column", false));
    ECC_HIP(launch_grad_filter_cols(st, c3, batch, Bk, pBk, pBi, Px, Gh, pG, W, D, pD, Px, ny, Py, Px, U,
                                    g.Ty->desc, g.Ty->f()));
    ColCfg c4 = col_config(*g.Ty, 3, sizeof(cx<float>), 256);
    RowCfg r5 = row_config(*g.Tx, Px, sizeof(cx<float>));
    ECC_TRY(check_cfg_col(c4, *g.Ty, sizeof(cx<float>), "column", false));
    ECC_TRY(check_cfg_row(r5, *g.Tx, sizeof(cx<float>), "row"));
    ECC_HIP((launch_fft_cols<float>(st, c4, U, +1, D, pD, Px, Px, Py, 0, Ts, (long long)Sz * Px, Px, Sz,
                                    -R, g.Ty->desc, g.Ty->f())));
    ECC_HIP((launch_fft_rows<float>(st, r5, U, +1, Ts, (long long)Sz * Px, Px, Sz, Px, 0, win,
                                    (long long)Sz * Sz, Sz, Sz, -R, g.Tx->desc, g.Tx->f())));
    ECC_HIP(launch_grad_filter_finish(st, win, (long long)Sz * Sz, Sz, plan->d_weights.as<float>(), scl,
                                      reinterpret_cast<cx<float>*>(grad_comps), Sz, U));
  }
  return ECC_OK;
}

}  // extern "C"

// =====================================================================================
// Workspace sizing: the same strategy choice and size formulas as the calls themselves.
namespace {

ecc_status workspace_need(ecc_context ctx, int call, ecc_filter_plan plan, int batch, int ny, int nx,
                          size_t* bytes) {
  const int R = plan->R, U = plan->U, Sz = plan->S;
  const int Py = fft_size_for(ctx, ny, R), Px = fft_size_for(ctx, nx, R);
  auto strat = [&](ecc_op op, int b, TileChoice& tc, bool* tiled, bool allow_direct = false) -> ecc_status {
    ecc_strategy used = ECC_STRATEGY_TWO_PASS;
    ECC_TRY(resolve_strategy(ctx, op, plan, ny, nx, b, &used, &tc, allow_direct));
    *tiled = used == ECC_STRATEGY_TILED || used == ECC_STRATEGY_DIRECT;   // neither takes workspace
    return ECC_OK;
  };
  // the signal/field part of the convolution adjoint, and the field part of the
  // correlation adjoint: an on-chip correlation with a second output, or the stack
  auto corr_y2 = [&](size_t* n) -> ecc_status {
    TileChoice tc;
    bool tiled = false;
    ECC_TRY(strat(ECC_CORRELATION, batch, tc, &tiled));
    *n = (tiled && tile_has_y2(tc.N, tc.TV)) ? 0 : ws_corr_stack(batch, ny, Py, Px, U);
    return ECC_OK;
  };
  auto gradf = [&](size_t* n) -> ecc_status {
    TileChoice tc;
    bool tiled = false;
    ECC_TRY(strat(ECC_CONVOLUTION, batch, tc, &tiled));
    if (tiled && tgradf_supported(tc.N, tc.TV)) {
      const long long nblk = (long long)((ny + tc.T - 1) / tc.T) * ((nx + tc.T - 1) / tc.T) * batch;
      *n = ws_gradf_parts(nblk, U, Sz) + gradf_reduce_scratch(U, Sz);
    } else {
      *n = ws_gradf_two_pass(batch, ny, Py, Px, U, Sz, false);
    }
    return ECC_OK;
  };
  TileChoice tc;
  bool tiled = false;
  size_t a = 0, b = 0, c = 0;
  switch (call) {
    case ECC_WS_EXTENDED_CORRELATION:
      ECC_TRY(strat(ECC_CORRELATION, batch, tc, &tiled, true));
      *bytes = tiled ? 0 : ws_corr_stack(batch, ny, Py, Px, U);
      return ECC_OK;
    case ECC_WS_EXTENDED_CONVOLUTION: {
      ECC_TRY(strat(ECC_CONVOLUTION, batch, tc, &tiled, true));
      TileChoice rc;
      if (tiled && tc.N == 128 && pick_tile_ratio(plan, rc))
        *bytes = tratio_scratch_bytes(rc.N, rc.T, batch, ny, nx);
      else *bytes = tiled ? 0 : ws_conv_two_pass(batch, ny, Py, Px, U, 1, false);
      return ECC_OK;
    }
    case ECC_WS_SCALE_SMOOTH:
    case ECC_WS_NORMALIZED_CONVOLUTION: {
      if (call == ECC_WS_SCALE_SMOOTH) {
        ECC_REQ(plan->group == ECC_GROUP_SCALE, "scale smoothing needs a scale plan");
        ECC_REQ(batch == 1, "scale smoothing takes one image");
      }
      ECC_TRY(strat(ECC_CONVOLUTION, batch, tc, &tiled));
      TileChoice rc;
      if (tiled && tc.N == 128 && pick_tile_ratio(plan, rc))
        *bytes = tratio_scratch_bytes(rc.N, rc.T, batch, ny, nx);
      else *bytes = tiled ? 0 : ws_conv_two_pass(batch, ny, Py, Px, U, 2, false);
      return ECC_OK;
    }
    case ECC_WS_JOINT_CONVOLUTION:
      ECC_TRY(strat(ECC_CONVOLUTION, batch, tc, &tiled));
      *bytes = tiled ? 0 : ws_conv_two_pass(batch, ny, Py, Px, U, 2, false);
      return ECC_OK;
    case ECC_WS_MATCH_ROTATIONS:
      ECC_REQ(batch == 1, "matching takes one image");
      ECC_TRY(strat(ECC_CORRELATION, 1, tc, &tiled));
      *bytes = tiled ? ws_match_tiled(ny, nx, U) : ws_corr_stack(1, ny, Py, Px, U);
      return ECC_OK;
    case ECC_WS_BACKWARD_CONVOLUTION:
      ECC_TRY(corr_y2(&a));
      ECC_TRY(gradf(&b));
      *bytes = std::max(a, b);
      return ECC_OK;
    case ECC_WS_BACKWARD_CORRELATION:
      ECC_TRY(corr_y2(&a));
      ECC_TRY(strat(ECC_CONVOLUTION, batch, tc, &tiled));
      b = tiled ? 0 : ws_conv_two_pass(batch, ny, Py, Px, U, 1, false);
      ECC_TRY(gradf(&c));
      *bytes = std::max(a, std::max(b, c));
      return ECC_OK;
  }
  return fail(ECC_ERR_INVALID_ARGUMENT, "unknown call for ecc_workspace_size");
}

}  // namespace

extern "C" {

ecc_status ecc_workspace_size(ecc_context ctx, int call, ecc_filter_plan plan, int batch, int ny, int nx,
                              size_t* bytes) {
  ECC_REQ(ctx && plan && bytes, "NULL argument");
  ECC_REQ(plan->ctx == ctx, "plan belongs to another context");
  ECC_TRY(validate_images(plan, batch, ny, nx, call == ECC_WS_JOINT_CONVOLUTION));
  if (call == ECC_WS_BACKWARD_CONVOLUTION || call == ECC_WS_BACKWARD_CORRELATION)
    ECC_REQ(plan->group == ECC_GROUP_ROTATION, "the adjoint needs a rotation plan");
  if (call == ECC_WS_MATCH_ROTATIONS) ECC_REQ(plan->group == ECC_GROUP_ROTATION, "matching needs a rotation plan");
  DeviceGuard dg(ctx->device);
  if (ctx->autotune) ECC_TRY(calibrate_tiles(ctx, nullptr));
  return workspace_need(ctx, call, plan, batch, ny, nx, bytes);
}

ecc_status ecc_workspace_reserve(ecc_context ctx, size_t bytes) {
  ECC_REQ(ctx, "NULL context");
  DeviceGuard dg(ctx->device);
  ECC_HIP(ctx->ws.ensure(bytes));
  return ECC_OK;
}

ecc_status ecc_workspace_allocated(ecc_context ctx, size_t* bytes) {
  ECC_REQ(ctx && bytes, "NULL argument");
  *bytes = ctx->ws.n;
  return ECC_OK;
}

}  // extern "C"
