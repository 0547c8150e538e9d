// Batches of independent extended correlations (many images, filters and band limits of
// different sizes) run as a few captured kernel launches, and the block-shape chooser of
// the tiled path with its on-device calibration.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "api_common.hpp"

using namespace ecc;

namespace ecc {
namespace {

// compiled block shapes (N, TV) of the tiled path
const int kShapes[][2] = {{64, 64}, {96, 64}, {128, 64}, {128, 96}};

int cu_count(ecc_context ctx) {
  if (ctx->num_cus <= 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || n <= 0)
      n = 256;
    ctx->num_cus = n;
  }
  return ctx->num_cus;
}

int blocks_per_cu(ecc_context ctx, int N, int TV) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, int> cache;
  std::lock_guard<std::mutex> g(mu);
  auto key = std::make_pair(N, TV);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  DeviceGuard dg(ctx->device);
  const int v = tile_blocks_per_cu(N, TV);
  cache[key] = v;
  return v;
}

}  // namespace

bool pick_tile(ecc_context ctx, int R, int U, int ny, int nx, int batch, bool throughput, int min_T,
               TileChoice& best) {
  bool found = false;
  const int cus = cu_count(ctx);
  for (const auto& c : kShapes) {
    const int N = c[0], TV = c[1];
    if (!tile_supported(N, TV)) continue;
    const int T = std::min(TV, N - 2 * R);
    if (T < std::max(16, min_T)) continue;
    const int per_cu = blocks_per_cu(ctx, N, TV);
    const double blocks = (double)((ny + T - 1) / T) * (double)((nx + T - 1) / T) * batch;
    const double slots = (double)cus * per_cu;
    const double waves = throughput ? blocks / slots : std::ceil(blocks / slots);
    double wave_cost;
    auto it = ctx->tile_cost.find({N, TV});
    if (ctx->tile_calibrated && it != ctx->tile_cost.end()) {
      wave_cost = it->second.a + it->second.b * U;   // measured (ms per wave)
    } else {
      // operation count: per block and component N column + T row transforms of length
      // N; the blocks sharing a CU share its arithmetic units
      wave_cost = (double)N * (N + T) * std::log2((double)N) * per_cu * (1.0 + U);
    }
    const double cost = waves * wave_cost;
    if (!found || cost < best.cost) {
      best.N = N;
      best.TV = TV;
      best.T = T;
      best.cost = cost;
      found = true;
    }
  }
  return found;
}

// Time per output pixel of the two forms, fitted to one MI355X (2048^2 images, S = 3..15,
// K = 1..16). Correlation: the direct sums about 4.2 ps + 0.0545 ps per component and tap
// (two FMAs at ~93% of the non-packed FP32 rate), the block path with the 64-point blocks
// that small filters take about 6.6 ps + 1.6 ps per component. Convolution: 4.8 + 0.0553
// per component and tap against 7.85 + 1.84 per component. Smaller images favour the
// direct form further (the block path's last wave of blocks is partly empty), so the
// comparison is made at the per-pixel rates alone.
bool direct_preferred(ecc_context ctx, bool conv, int S, int U, int ny, int nx, int batch) {
  (void)ctx;
  (void)ny;
  (void)nx;
  (void)batch;
  const double taps = (double)U * S * S;
  const double direct_ps = conv ? 4.8 + 0.0553 * taps : 4.2 + 0.0545 * taps;
  const double blocks_ps = conv ? 7.85 + 1.84 * U : 6.6 + 1.6 * U;
  return direct_ps < blocks_ps;
}

bool pick_tile_conv(ecc_context ctx, int R, int U, int ny, int nx, int batch, int min_T, TileChoice& best) {
  bool found = false;
  const int cus = cu_count(ctx);
  for (const auto& c : kShapes) {
    const int N = c[0], TV = c[1];
    if (!tconv_supported(N, TV)) continue;
    const int T = std::min(TV, N - 2 * R);
    if (T < std::max(16, min_T)) continue;
    const double blocks = (double)((ny + T - 1) / T) * (double)((nx + T - 1) / T) * batch;
    // per block and component 2N forward transforms of length N, one workgroup per CU
    const double cost = std::ceil(blocks / cus) * (double)N * (2 * N) * std::log2((double)N) * (1.0 + U);
    if (!found || cost < best.cost) {
      best.N = N;
      best.TV = TV;
      best.T = T;
      best.cost = cost;
      found = true;
    }
  }
  return found;
}

bool pick_tile_ratio(ecc_filter_plan plan, TileChoice& best) {
  if (!plan->symmetric || (int)plan->parity.size() != plan->U) return false;
  bool found = false;
  for (const auto& c : kShapes) {
    const int N = c[0], TV = c[1];
    if (!tratio_supported(N, TV)) continue;
    const int T = std::min(TV, N - 2 * plan->R);
    if (T < 16) continue;
    const double cost = (double)N * N * std::log2((double)N) / ((double)T * T);
    if (!found || cost < best.cost) {
      best.N = N;
      best.TV = TV;
      best.T = T;
      best.cost = cost;
      found = true;
    }
  }
  return found;
}

ecc_status calibrate_tiles(ecc_context ctx, hipStream_t st) {
  if (ctx->tile_calibrated) return ECC_OK;
  DeviceGuard dg(ctx->device);
  const int cus = cu_count(ctx);
  const int R = 3;           // any radius leaves the per-block work unchanged
  const int Ulo = 2, Uhi = 8;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ECC_HIP(hipEventCreate(&e0));
  ECC_HIP(hipEventCreate(&e1));
  ecc_status status = ECC_OK;
  for (const auto& c : kShapes) {
    const int N = c[0], TV = c[1];
    if (!tile_supported(N, TV)) continue;
    const int T = std::min(TV, N - 2 * R);
    const int per_cu = blocks_per_cu(ctx, N, TV);
    const long long slots = (long long)cus * per_cu;
    const int side = (int)std::ceil(std::sqrt(2.0 * (double)slots));   // >= 2 full waves
    const int n = side * T;
    const double waves = std::ceil((double)side * side / (double)slots);
    DevBuf img, fld, out, spec, w;
    hipError_t e = img.ensure((size_t)n * n * sizeof(float));
    if (e == hipSuccess) e = fld.ensure((size_t)n * n * sizeof(float));
    if (e == hipSuccess) e = out.ensure((size_t)n * n * sizeof(float));
    if (e == hipSuccess) e = spec.ensure((size_t)Uhi * N * N * sizeof(cx<float>));
    if (e == hipSuccess) e = w.ensure(Uhi * sizeof(float));
    if (e == hipSuccess) e = hipMemsetAsync(img.p, 0, (size_t)n * n * sizeof(float), st);
    if (e == hipSuccess) e = hipMemsetAsync(fld.p, 0, (size_t)n * n * sizeof(float), st);
    if (e == hipSuccess) e = hipMemsetAsync(spec.p, 0, (size_t)Uhi * N * N * sizeof(cx<float>), st);
    if (e == hipSuccess) e = hipMemsetAsync(w.p, 0, Uhi * sizeof(float), st);
    Field fl{fld.as<float>(), 0, n, 0, 1.0, 0.0};
    double best[2] = {1e30, 1e30};
    for (int u = 0; u < 2 && e == hipSuccess; ++u) {
      const int U = u ? Uhi : Ulo;
      for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {   // first run warms up
        e = hipEventRecord(e0, st);
        if (e == hipSuccess)
          e = launch_tile_corr(st, N, TV, 1, img.as<float>(), 0, n, fl, out.as<float>(), 0, n, n, n, R, T, U,
                               0, w.as<float>(), 1.f, spec.as<cx<float>>());
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && rep > 0) best[u] = std::min(best[u], (double)ms / waves);
      }
    }
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(st);
      status = fail(ECC_ERR_HIP, std::string("block-shape calibration: ") + hipGetErrorString(e));
      break;
    }
    ecc_context_s::TileCost tcost;
    tcost.b = std::max(0.0, (best[1] - best[0]) / (Uhi - Ulo));
    tcost.a = std::max(0.0, best[0] - Ulo * tcost.b);
    ctx->tile_cost[{N, TV}] = tcost;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status == ECC_OK) ctx->tile_calibrated = true;
  return status;
}

}  // namespace ecc

// =====================================================================================
struct ecc_batch_plan_s {
  ecc_context ctx = nullptr;
  int flags = 0;
  std::vector<ecc_instance> inst;
  struct Shape {
    int N = 0, TV = 0, nwg = 0, nitems = 0;
    bool sym = false;                // symmetric form (centred spectra)
    bool conv = false;               // convolutions (block convolution, item table)
    bool direct = false;             // direct correlations (N holds the filter side)
    std::vector<int> members;        // instance indices, in descriptor order
    std::vector<int> T;              // block side per member
    DevBuf descs, items, ctr;        // ctr: the persistent form's counter pair
  };
  std::deque<Shape> shapes;         // deque: elements own device buffers and never move
  std::vector<int> rest;             // instances for the per-call path
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;         // recorded after every execution's last launch
  // capture-time fork/join: one stream and one event per block shape, so that the
  // graph holds the shapes' launches as parallel branches and their tails overlap
  std::vector<hipStream_t> branch;
  std::vector<hipEvent_t> joined;
  hipEvent_t fork = nullptr;
  int nblocks = 0;
  ~ecc_batch_plan_s() {
    for (hipEvent_t e : joined) (void)hipEventDestroy(e);
    for (hipStream_t b : branch) (void)hipStreamDestroy(b);
    if (fork) (void)hipEventDestroy(fork);
    if (done) (void)hipEventDestroy(done);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

namespace {

ecc_status check_instance(ecc_context ctx, const ecc_instance& in) {
  ECC_REQ(in.plan && in.plan->ctx == ctx, "instance plan is NULL or belongs to another context");
  ECC_REQ(in.op == ECC_CORRELATION || in.op == ECC_CONVOLUTION, "unknown op");
  ECC_REQ(in.signal && in.field && in.out, "NULL image pointer");
  ECC_TRY(validate_images(in.plan, 1, in.ny, in.nx));
  ECC_REQ(in.ld_signal >= in.nx && in.ld_field >= in.nx && in.ld_out >= in.nx, "row strides must be >= nx");
  const size_t bo = (size_t)in.ny * in.ld_out * sizeof(float);
  ECC_REQ(!overlaps(in.out, bo, in.signal, (size_t)in.ny * in.ld_signal * sizeof(float)) &&
              !overlaps(in.out, bo, in.field, (size_t)in.ny * in.ld_field * sizeof(float)),
          "out aliases an input");
  return ECC_OK;
}

TileArgs make_desc(const ecc_instance& in, int N, int T, const Spectrum* sp) {
  TileArgs a{};
  a.H = in.signal;
  a.planeH = 0;
  a.ldH = in.ld_signal;
  a.fld = make_field(in.plan, in.field, 0, in.ld_field, 1.0);
  a.y = in.out;
  a.planeY = 0;
  a.ldY = in.ld_out;
  a.ny = in.ny;
  a.nx = in.nx;
  a.R = in.plan->R;
  a.T = T;
  a.tx = (in.nx + T - 1) / T;
  a.ty = (in.ny + T - 1) / T;
  a.U = in.plan->U;
  a.kofs = 0;
  a.w = in.plan->d_weights.as<float>();
  a.scale = 1.0f / ((float)N * (float)N);
  a.Fs = sp->buf.as<cx<float>>();
  return a;
}

TileConvArgs make_conv_desc(const ecc_instance& in, int N, int T, const Spectrum* sp) {
  TileConvArgs a{};
  a.H = in.signal;
  a.planeH = 0;
  a.ldH = in.ld_signal;
  a.fld = make_field(in.plan, in.field, 0, in.ld_field, 1.0);
  a.sig_norm = 0;
  a.nsig = 1;
  a.step = 0;
  a.y = in.out;
  a.planeY = 0;
  a.ldY = in.ld_out;
  a.ny = in.ny;
  a.nx = in.nx;
  a.R = in.plan->R;
  a.T = T;
  a.tx = (in.nx + T - 1) / T;
  a.ty = (in.ny + T - 1) / T;
  a.U = in.plan->U;
  a.w = in.plan->d_weights.as<float>();
  a.scale = 1.0f / ((float)N * (float)N);
  a.Fs = sp->buf.as<cx<float>>();
  return a;
}

ecc_status upload_descs(ecc_batch_plan bp, hipStream_t st) {
  for (auto& sh : bp->shapes) {
    if (sh.conv && !sh.direct) {
      std::vector<TileConvArgs> d;
      for (size_t m = 0; m < sh.members.size(); ++m) {
        const ecc_instance& in = bp->inst[sh.members[m]];
        const Spectrum* sp = nullptr;
        ECC_TRY(get_tile_spectrum(in.plan, sh.N, st, &sp, SPEC_CONV));
        d.push_back(make_conv_desc(in, sh.N, sh.T[m], sp));
      }
      ECC_HIP(sh.descs.ensure(d.size() * sizeof(TileConvArgs)));
      ECC_HIP(hipMemcpy(sh.descs.p, d.data(), d.size() * sizeof(TileConvArgs), hipMemcpyHostToDevice));
      continue;
    }
    std::vector<TileArgs> d;
    for (size_t m = 0; m < sh.members.size(); ++m) {
      const ecc_instance& in = bp->inst[sh.members[m]];
      if (sh.direct) {
        TileArgs a{};
        a.H = in.signal;
        a.ldH = in.ld_signal;
        a.fld = make_field(in.plan, in.field, 0, in.ld_field, 1.0);
        a.y = in.out;
        a.ldY = in.ld_out;
        a.ny = in.ny;
        a.nx = in.nx;
        a.R = in.plan->R;
        direct_blocks(in.ny, in.nx, &a.tx, &a.ty);
        a.U = in.plan->U;
        a.w = in.plan->d_weights.as<float>();
        a.scale = 1.0f;
        a.Fs = in.plan->comps32.as<cx<float>>();
        d.push_back(a);
        continue;
      }
      const Spectrum* sp = nullptr;
      ECC_TRY(get_tile_spectrum(in.plan, sh.N, st, &sp, sh.sym ? SPEC_CENTRED : SPEC_CORR));
      d.push_back(make_desc(in, sh.N, sh.T[m], sp));
      d.back().sym = sh.sym ? 1 : 0;
    }
    ECC_HIP(sh.descs.ensure(d.size() * sizeof(TileArgs)));
    ECC_HIP(hipMemcpy(sh.descs.p, d.data(), d.size() * sizeof(TileArgs), hipMemcpyHostToDevice));
  }
  return ECC_OK;
}

}  // namespace

extern "C" {

ecc_status ecc_batch_plan_create(ecc_context ctx, const ecc_instance* inst, int n, int flags,
                                 ecc_batch_plan* out) {
  ECC_REQ(ctx && out, "NULL argument");
  *out = nullptr;
  ECC_REQ(n >= 0 && n <= (1 << 20) && (n == 0 || inst), "bad instance list");
  ECC_REQ((flags & ~(ECC_BATCH_AUTOTUNE | ECC_BATCH_PERSISTENT)) == 0, "unknown flags");
  for (int i = 0; i < n; ++i) ECC_TRY(check_instance(ctx, inst[i]));
  DeviceGuard dg(ctx->device);
  auto bp = std::make_unique<ecc_batch_plan_s>();
  bp->ctx = ctx;
  bp->flags = flags;
  bp->inst.assign(inst, inst + n);
  ECC_HIP(hipStreamCreateWithFlags(&bp->cs, hipStreamNonBlocking));
  ECC_HIP(hipEventCreateWithFlags(&bp->done, hipEventDisableTiming));
  if (flags & ECC_BATCH_AUTOTUNE) ECC_TRY(calibrate_tiles(ctx, bp->cs));

  // ---- block shape and form per instance (the shapes the per-call path would take)
  std::map<std::tuple<int, int, bool, bool, bool>, int> shape_of;
  for (int i = 0; i < n; ++i) {
    const ecc_instance& in = inst[i];
    TileChoice tc;
    const int R = in.plan->R, S = in.plan->S, U = in.plan->U;
    const bool conv = in.op == ECC_CONVOLUTION;
    // direct sums: forced (DIRECT strategy, any instance with a kernel for its side) or
    // chosen by the same time model as a single call (AUTO)
    const bool direct = direct_supported(S) &&
                        (ctx->strategy == ECC_STRATEGY_DIRECT ||
                         (ctx->strategy == ECC_STRATEGY_AUTO && direct_preferred(ctx, conv, S, U, in.ny, in.nx, 1)));
    const ecc_strategy want = ctx->strategy == ECC_STRATEGY_DIRECT ? ECC_STRATEGY_AUTO : ctx->strategy;
    const int min_T = want == ECC_STRATEGY_AUTO ? 2 * R : 16;
    const bool tiled = direct || (want != ECC_STRATEGY_TWO_PASS &&
                                  (conv ? pick_tile_conv(ctx, R, U, in.ny, in.nx, 1, min_T, tc)
                                        : pick_tile(ctx, R, U, in.ny, in.nx, 1, true, min_T, tc)));
    if (!tiled) {
      bp->rest.push_back(i);
      continue;
    }
    if (direct) {
      tc.N = S;
      tc.TV = 0;
      tc.T = 0;
    }
    const bool sym = !conv && !direct && tile_symmetric(tc.N, tc.TV) && rotation_parity(in.plan);
    auto key = std::make_tuple(tc.N, tc.TV, sym, conv, direct);
    auto it = shape_of.find(key);
    if (it == shape_of.end()) {
      it = shape_of.emplace(key, (int)bp->shapes.size()).first;
      bp->shapes.emplace_back();
      bp->shapes.back().N = tc.N;
      bp->shapes.back().TV = tc.TV;
      bp->shapes.back().sym = sym;
      bp->shapes.back().conv = conv;
      bp->shapes.back().direct = direct;
    }
    bp->shapes[it->second].members.push_back(i);
    bp->shapes[it->second].T.push_back(tc.T);
  }
  ECC_TRY(upload_descs(bp.get(), bp->cs));

  // ---- block lists, longest first
  const int cus = cu_count(ctx);
  for (auto& sh : bp->shapes) {
    struct Item {
      int desc, block, cost;
    };
    std::vector<Item> items;
    for (size_t m = 0; m < sh.members.size(); ++m) {
      const ecc_instance& in = inst[sh.members[m]];
      int nb;
      if (sh.direct) {
        int tx, ty;
        direct_blocks(in.ny, in.nx, &tx, &ty);
        nb = tx * ty;
      } else {
        const int T = sh.T[m];
        nb = ((in.ny + T - 1) / T) * ((in.nx + T - 1) / T);
      }
      for (int b = 0; b < nb; ++b) items.push_back({(int)m, b, in.plan->U});
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
    sh.nitems = (int)items.size();
    bp->nblocks += sh.nitems;
    std::vector<int2> list;
    for (const Item& it : items) list.push_back(make_int2(it.desc, it.block));
    sh.nwg = sh.nitems;
    if ((flags & ECC_BATCH_PERSISTENT) && !sh.conv && !sh.direct) {
      // as many workgroups as fit at once; they draw the items, longest first, from the
      // counter pair (zero now, and zero again after every launch)
      sh.nwg = std::max(1, std::min<int>(sh.nitems, cus * blocks_per_cu(ctx, sh.N, sh.TV)));
      ECC_HIP(sh.ctr.ensure(2 * sizeof(int)));
      ECC_HIP(hipMemset(sh.ctr.p, 0, 2 * sizeof(int)));
    }
    ECC_HIP(sh.items.ensure(std::max<size_t>(1, list.size()) * sizeof(int2)));
    if (!list.empty()) ECC_HIP(hipMemcpy(sh.items.p, list.data(), list.size() * sizeof(int2), hipMemcpyHostToDevice));
  }

  // ---- capture the launches once
  bool any = false;
  for (auto& sh : bp->shapes) any = any || sh.nitems > 0;
  if (any) {
    ECC_HIP(hipEventCreateWithFlags(&bp->fork, hipEventDisableTiming));
    for (auto& sh : bp->shapes) {
      if (sh.nitems == 0) continue;
      bp->branch.push_back(nullptr);
      ECC_HIP(hipStreamCreateWithFlags(&bp->branch.back(), hipStreamNonBlocking));
      bp->joined.push_back(nullptr);
      ECC_HIP(hipEventCreateWithFlags(&bp->joined.back(), hipEventDisableTiming));
    }
    ECC_HIP(hipStreamBeginCapture(bp->cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipEventRecord(bp->fork, bp->cs);
    size_t b = 0;
    for (auto& sh : bp->shapes) {
      if (sh.nitems == 0 || e != hipSuccess) continue;
      hipStream_t st = bp->branch[b];
      e = hipStreamWaitEvent(st, bp->fork, 0);
      if (e == hipSuccess)
        e = sh.direct ? launch_direct_items(st, sh.conv, sh.N, sh.descs.as<TileArgs>(), sh.items.as<int2>(),
                                            sh.nitems)
            : sh.conv ? launch_tile_conv_items(st, sh.N, sh.TV, sh.descs.as<TileConvArgs>(), sh.items.as<int2>(),
                                               sh.nitems)
                        : launch_tile_batch(st, sh.N, sh.TV, sh.sym, sh.nwg, sh.descs.as<TileArgs>(),
                                            sh.items.as<int2>(), sh.nitems,
                                            (flags & ECC_BATCH_PERSISTENT) ? sh.ctr.as<int>() : nullptr);
      if (e == hipSuccess) e = hipEventRecord(bp->joined[b], st);
      if (e == hipSuccess) e = hipStreamWaitEvent(bp->cs, bp->joined[b], 0);
      ++b;
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(bp->cs, &g);
    bp->graph = g;
    ECC_HIP(e);
    ECC_HIP(e2);
    ECC_HIP(hipGraphInstantiate(&bp->exec, bp->graph, nullptr, nullptr, 0));
  }
  *out = bp.release();
  return ECC_OK;
}

ecc_status ecc_batch_update(ecc_batch_plan bp, const ecc_instance* inst, int n) {
  ECC_REQ(bp && (n == 0 || inst), "NULL argument");
  ECC_REQ(n == (int)bp->inst.size(), "instance count differs from the plan");
  for (int i = 0; i < n; ++i) {
    const ecc_instance& a = inst[i];
    const ecc_instance& b = bp->inst[i];
    ECC_REQ(a.op == b.op && a.plan == b.plan && a.ny == b.ny && a.nx == b.nx,
            "instance op, plan or size differs from the plan");
    ECC_TRY(check_instance(bp->ctx, a));
  }
  DeviceGuard dg(bp->ctx->device);
  // the descriptors are rewritten in place: wait for the last execution (on whatever
  // stream it ran) and for the upload stream
  ECC_HIP(hipEventSynchronize(bp->done));
  ECC_HIP(hipStreamSynchronize(bp->cs));
  bp->inst.assign(inst, inst + n);
  ECC_TRY(upload_descs(bp, bp->cs));
  return ECC_OK;
}

ecc_status ecc_batch_execute(ecc_batch_plan bp, void* stream) {
  ECC_REQ(bp, "NULL batch plan");
  DeviceGuard dg(bp->ctx->device);
  hipStream_t st = S(stream);
  if (bp->exec) ECC_HIP(hipGraphLaunch(bp->exec, st));
  for (int i : bp->rest) {
    const ecc_instance& in = bp->inst[i];
    ECC_TRY(forward_impl(bp->ctx, in.op, in.plan, 1, in.ny, in.nx, in.signal, in.ld_signal, in.field,
                         in.ld_field, in.out, in.ld_out, st, nullptr));
  }
  ECC_HIP(hipEventRecord(bp->done, st));
  return ECC_OK;
}

ecc_status ecc_batch_info(ecc_batch_plan bp, int* graph_instances, int* launches, int* blocks) {
  ECC_REQ(bp, "NULL batch plan");
  int gi = 0, nl = 0;
  for (auto& sh : bp->shapes) {
    gi += (int)sh.members.size();
    nl += sh.nitems > 0 ? 1 : 0;
  }
  if (graph_instances) *graph_instances = gi;
  if (launches) *launches = nl;
  if (blocks) *blocks = bp->nblocks;
  return ECC_OK;
}

ecc_status ecc_batch_plan_destroy(ecc_batch_plan bp) {
  if (!bp) return ECC_OK;
  DeviceGuard dg(bp->ctx->device);
  if (bp->cs) (void)hipStreamSynchronize(bp->cs);
  (void)hipDeviceSynchronize();
  delete bp;
  return ECC_OK;
}


namespace {
// the device's architecture name ("gfx950:sramecc+:xnack-"), which the costs belong to
std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  return std::string(prop.gcnArchName);
}
}  // namespace

ecc_status ecc_autotune_export(ecc_context ctx, char* buf, size_t cap, size_t* len) {
  ECC_REQ(ctx && len, "NULL argument");
  ECC_REQ(ctx->tile_calibrated, "the context has not calibrated its block shapes yet");
  std::string j = "{\"device\": \"" + arch_name(ctx->device) + "\", \"tile_cost\": [";
  bool first = true;
  for (const auto& kv : ctx->tile_cost) {
    char item[128];
    std::snprintf(item, sizeof(item), "%s[%d, %d, %.9g, %.9g]", first ? "" : ", ", kv.first.first, kv.first.second,
                  kv.second.a, kv.second.b);
    j += item;
    first = false;
  }
  j += "], \"fft_size\": [";
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    first = true;
    for (const auto& kv : ctx->tuned) {
      int n = 0, R = 0;
      if (std::sscanf(kv.first.c_str(), "%d:%d", &n, &R) != 2) continue;
      char item[64];
      std::snprintf(item, sizeof(item), "%s[%d, %d, %d]", first ? "" : ", ", n, R, kv.second);
      j += item;
      first = false;
    }
  }
  j += "]}";
  *len = j.size();
  if (buf) {
    ECC_REQ(cap > j.size(), "buffer too small (see *len)");
    std::memcpy(buf, j.c_str(), j.size() + 1);
  }
  return ECC_OK;
}

ecc_status ecc_autotune_import(ecc_context ctx, const char* json) {
  ECC_REQ(ctx && json, "NULL argument");
  const std::string j(json);
  const std::string dkey = "\"device\": \"";
  const size_t d0 = j.find(dkey);
  ECC_REQ(d0 != std::string::npos, "no device name in the autotuner text");
  const size_t d1 = j.find('"', d0 + dkey.size());
  ECC_REQ(d1 != std::string::npos, "unterminated device name");
  ECC_REQ(j.substr(d0 + dkey.size(), d1 - d0 - dkey.size()) == arch_name(ctx->device),
          "the autotuner text was measured on another kind of device");
  const size_t t0 = j.find("\"tile_cost\"", d1);
  ECC_REQ(t0 != std::string::npos, "no tile_cost in the autotuner text");
  size_t pos = j.find('[', t0);
  ECC_REQ(pos != std::string::npos, "malformed tile_cost");
  std::map<std::pair<int, int>, ecc_context_s::TileCost> costs;
  ++pos;
  while (true) {
    const size_t open = j.find('[', pos), close = j.find(']', pos);
    ECC_REQ(close != std::string::npos, "malformed tile_cost");
    if (open == std::string::npos || open > close) break;   // the list's closing bracket
    int N = 0, TV = 0;
    double a = 0, b = 0;
    ECC_REQ(std::sscanf(j.c_str() + open, "[%d , %d , %lf , %lf ]", &N, &TV, &a, &b) == 4,
            "malformed tile_cost entry");
    ECC_REQ(tile_supported(N, TV) && std::isfinite(a) && std::isfinite(b) && a >= 0 && b >= 0,
            "tile_cost entry for an unknown block shape or with a negative cost");
    ecc_context_s::TileCost tc;
    tc.a = a;
    tc.b = b;
    costs[{N, TV}] = tc;
    pos = j.find(']', open) + 1;
  }
  for (const auto& c : kShapes)
    if (tile_supported(c[0], c[1]))
      ECC_REQ(costs.count({c[0], c[1]}), "the autotuner text lacks a block shape this library has");
  // two-pass FFT sizes chosen by the autotuner (optional): [n, R, P] with P a 7-smooth size
  // at least the smallest admissible one
  std::map<std::string, int> sizes;
  const size_t f0 = j.find("\"fft_size\"");
  if (f0 != std::string::npos) {
    size_t fp = j.find('[', f0);
    ECC_REQ(fp != std::string::npos, "malformed fft_size");
    ++fp;
    while (true) {
      const size_t open = j.find('[', fp), close = j.find(']', fp);
      ECC_REQ(close != std::string::npos, "malformed fft_size");
      if (open == std::string::npos || open > close) break;
      int n = 0, R = 0, P = 0;
      ECC_REQ(std::sscanf(j.c_str() + open, "[%d , %d , %d ]", &n, &R, &P) == 3, "malformed fft_size entry");
      ECC_REQ(n >= 1 && R >= 0 && P >= n + R && P >= 2 * R + 1 && P >= 16 && next_smooth7(P) == P && P <= 16384,
              "fft_size entry out of range");
      sizes[std::to_string(n) + ":" + std::to_string(R)] = P;
      fp = j.find(']', open) + 1;
    }
  }
  ctx->tile_cost = costs;
  ctx->tile_calibrated = true;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    for (const auto& kv : sizes) ctx->tuned[kv.first] = kv.second;
  }
  return ECC_OK;
}

}  // extern "C"
