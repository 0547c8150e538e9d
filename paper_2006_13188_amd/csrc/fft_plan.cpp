// Host-side planning of the LDS transforms: 7-smooth size selection, radix schedules,
// float64 twiddle tables (stored as float64 and rounded to float32), launch geometry.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <functional>

namespace ecc {

static bool factor7(int n, std::vector<int>& primes) {
  primes.clear();
  for (int p : {7, 5, 3, 2}) {
    while (n % p == 0) {
      primes.push_back(p);
      n /= p;
    }
  }
  return n == 1;
}

bool is_smooth7(int n) {
  std::vector<int> p;
  return n >= 1 && factor7(n, p);
}

int next_smooth7(int n) {
  for (int m = std::max(n, 1);; ++m)
    if (is_smooth7(m)) return m;
}

// Fewest passes with radices in [2, 8] (the butterflies the LDS engine instantiates);
// ties go to the schedule with the largest smallest radix (fewer butterflies per
// thread in the worst pass).
std::vector<int> choose_radices(int P) {
  std::vector<int> primes;
  if (!factor7(P, primes)) return {};
  if (P == 1) return {};
  std::vector<int> best;
  std::vector<int> groups;
  std::function<void(size_t)> dfs = [&](size_t i) {
    if (!best.empty() && groups.size() > best.size()) return;
    if (i == primes.size()) {
      std::vector<int> g = groups;
      std::sort(g.begin(), g.end(), std::greater<int>());
      if (best.empty() || g.size() < best.size() ||
          (g.size() == best.size() && g.back() > best.back()))
        best = g;
      return;
    }
    const int p = primes[i];
    for (size_t j = 0; j < groups.size(); ++j) {
      if (groups[j] * p <= 8) {
        groups[j] *= p;
        dfs(i + 1);
        groups[j] /= p;
      }
    }
    groups.push_back(p);
    dfs(i + 1);
    groups.pop_back();
  };
  dfs(0);
  return best;
}

static hipError_t make_transform(int P, Transform& t) {
  t.desc = FftDesc{};
  t.desc.P = P;
  std::vector<int> rad = choose_radices(P);
  if (rad.empty() || (int)rad.size() > kMaxPass) return hipErrorInvalidValue;
  t.desc.npass = (int)rad.size();
  std::vector<double> tw;
  int Ls = 1, off = 0;
  for (int p = 0; p < t.desc.npass; ++p) {
    const int R = rad[p];
    t.desc.radix[p] = R;
    t.desc.twoff[p] = off;
    t.desc.magic[p] = (Ls > 1) ? (uint32_t)((1ull << 32) / (unsigned long long)Ls + 1ull) : 0u;
    const long long N = (long long)Ls * R;
    for (int j = 0; j < Ls; ++j) {
      for (int r = 1; r < R; ++r) {
        // exp(-2 pi i r j / N), angle reduced exactly in integers, evaluated in long double
        long long m = ((long long)r * j) % N;
        if (2 * m > N) m -= N;
        const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)N;
        tw.push_back((double)cosl(a));
        tw.push_back((double)sinl(a));
      }
    }
    off += Ls * (R - 1);
    Ls *= R;
  }
  t.desc.twsize = off;
  t.rad = rad;
  const size_t n = std::max<size_t>(1, (size_t)off);
  std::vector<float> tw32(2 * n, 0.f);
  for (size_t i = 0; i < tw.size(); ++i) tw32[i] = (float)tw[i];
  std::vector<double> tw64(2 * n, 0.0);
  std::copy(tw.begin(), tw.end(), tw64.begin());
  hipError_t e = hipMalloc(&t.tw32, 2 * n * sizeof(float));
  if (e != hipSuccess) return e;
  e = hipMalloc(&t.tw64, 2 * n * sizeof(double));
  if (e != hipSuccess) return e;
  e = hipMemcpy(t.tw32, tw32.data(), 2 * n * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  e = hipMemcpy(t.tw64, tw64.data(), 2 * n * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  int R0 = 0, R1 = 0, R2 = 0;
  if (fixed_split(P, &R0, &R1, &R2)) {
    // pass 1: rows j < R0 of w1^{r j}, w1 = exp(-2 pi i / (R0 R1)), 1 <= r < R1;
    // pass 2: rows b < R0 R1 of w^{r b}, w = exp(-2 pi i / P), 1 <= r < R2
    std::vector<float> fx;
    auto put = [&](long long m, long long N) {
      m %= N;
      if (2 * m > N) m -= N;
      const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)N;
      fx.push_back((float)cosl(a));
      fx.push_back((float)sinl(a));
    };
    for (int j = 0; j < R0; ++j)
      for (int r = 1; r < R1; ++r) put((long long)r * j, (long long)R0 * R1);
    if (R2 > 1)
      for (int b = 0; b < R0 * R1; ++b)
        for (int r = 1; r < R2; ++r) put((long long)r * b, P);
    if (fx.empty()) fx.assign(2, 0.f);
    e = hipMalloc(&t.fx_tw32, fx.size() * sizeof(float));
    if (e != hipSuccess) return e;
    e = hipMemcpy(t.fx_tw32, fx.data(), fx.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    t.fR0 = R0;
    t.fR1 = R1;
    t.fR2 = R2;
  }
  return hipSuccess;
}

hipError_t get_transform(ecc_context_s* ctx, int P, const Transform** out) {
  std::lock_guard<std::mutex> g(ctx->mu);
  auto it = ctx->transforms.find(P);
  if (it != ctx->transforms.end()) {
    *out = it->second.get();
    return hipSuccess;
  }
  auto t = std::make_unique<Transform>();
  hipError_t e = make_transform(P, *t);
  if (e != hipSuccess) return e;
  *out = t.get();
  ctx->transforms[P] = std::move(t);
  return hipSuccess;
}

Transform::~Transform() {
  if (fx_tw32) (void)hipFree(fx_tw32);
  if (tw32) (void)hipFree(tw32);
  if (tw64) (void)hipFree(tw64);
}

int max_butterflies(const Transform& t) {
  int m = 0;
  for (int R : t.rad) m = std::max(m, t.desc.P / R);
  return m;
}

static int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Blocked row layout: TF threads per transform, B transforms per workgroup (<= 256
// threads), NB butterflies per thread per pass, EPX positions per thread over `span`.
RowCfg row_config(const Transform& t, int span, size_t elem, int max_threads) {
  const int nb = max_butterflies(t);
  RowCfg c{};
  const int TF = std::min(max_threads, std::max(32, pow2_at_least(nb)));
  c.TF = TF;
  c.NB = (nb <= TF) ? 1 : (nb <= 2 * TF ? 2 : (nb <= 4 * TF ? 4 : -1));
  c.B = std::max(1, 256 / TF);
  while (c.B > 1 && lds_rows(c, t.desc, elem) > 64 * 1024) c.B >>= 1;
  const int need = (span + TF - 1) / TF;
  c.EPX = need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : need <= 16 ? 16 : -1;
  // lines longer than max_threads can take (more than four butterflies or sixteen elements
  // per thread: lengths above 4096, or small radices above ~3000) get 512 threads, which
  // every row kernel accepts
  if ((c.NB < 0 || c.EPX < 0) && max_threads < 512) return row_config(t, span, elem, 512);
  return c;
}

// Interleaved column layout: 2^lgB adjacent columns, nthr threads. lgB is lowered from
// want_lgB until the butterflies per thread (NB <= 4) and the LDS (<= 150 KiB) fit.
ColCfg col_config(const Transform& t, int want_lgB, size_t elem, int nthr) {
  ColCfg c{};
  c.nthr = nthr;
  const int nb = max_butterflies(t);
  for (c.lgB = want_lgB; c.lgB >= 0; --c.lgB) {
    const int TF = nthr >> c.lgB;
    c.NB = (nb <= TF) ? 1 : (nb <= 2 * TF ? 2 : (nb <= 4 * TF ? 4 : -1));
    if (c.NB > 0 && lds_cols(c, t.desc, elem) <= 150 * 1024) break;
  }
  if (c.lgB < 0) {
    c.lgB = 0;
    c.NB = -1;
  }
  const int need = ((t.desc.P << c.lgB) + nthr - 1) / nthr;
  c.EPT = need <= 4 ? 4 : need <= 8 ? 8 : need <= 12 ? 12 : need <= 16 ? 16 : need <= 24 ? 24 : need <= 32 ? 32 : -1;
  return c;
}

}  // namespace ecc
