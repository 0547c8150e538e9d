// Helpers shared by the host-side translation units of libecc (api.cpp, batch.cpp):
// error reporting, device scoping, and the choice of block shapes for the tiled path.
#pragma once
#include <string>

#include "internal.hpp"

namespace ecc {

// Records `msg` as this thread's last error text and returns `s`.
ecc_status fail(ecc_status s, const std::string& msg);

#define ECC_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      if (e_ == hipErrorOutOfMemory)                                                   \
        return ::ecc::fail(ECC_ERR_OUT_OF_MEMORY, std::string(#expr) + ": out of memory"); \
      return ::ecc::fail(ECC_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    }                                                                                  \
  } while (0)

#define ECC_REQ(cond, msg)                                                   \
  do {                                                                       \
    if (!(cond)) return ::ecc::fail(ECC_ERR_INVALID_ARGUMENT, (msg));        \
  } while (0)

#define ECC_TRY(expr)                 \
  do {                                \
    ecc_status s_ = (expr);           \
    if (s_ != ECC_OK) return s_;      \
  } while (0)

// Makes the context's device current for one API call and clears any error state left
// behind by earlier HIP calls of the caller, so launch checks report this call's errors.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    (void)hipGetLastError();
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

inline hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

// Scope of one call's use of the context workspace on stream `st`: if the previous user
// ran on another stream, `st` first waits for its last kernel; on exit an event marks
// this call's last kernel. Calls from one host thread on several streams therefore never
// overwrite a workspace that queued work still reads.
struct WsUse {
  ecc_context ctx;
  hipStream_t st;
  WsUse(ecc_context c, hipStream_t s) : ctx(c), st(s) {
    if (ctx->ws_event && ctx->ws_stream != st) (void)hipStreamWaitEvent(st, ctx->ws_event, 0);
  }
  ~WsUse() {
    if (!ctx->ws_event && hipEventCreateWithFlags(&ctx->ws_event, hipEventDisableTiming) != hipSuccess)
      ctx->ws_event = nullptr;
    if (ctx->ws_event && hipEventRecord(ctx->ws_event, st) == hipSuccess) ctx->ws_stream = st;
  }
  WsUse(const WsUse&) = delete;
  WsUse& operator=(const WsUse&) = delete;
};

constexpr size_t kMaxLds = 160 * 1024;

// ---- tiled path
struct TileChoice {
  int N = 0, TV = 0, T = 0;
  double cost = 0;   // modelled time (see pick_tile)
};

// Block shape for a correlation with filter radius R and U components over `batch`
// images of ny x nx, among the shapes with block side >= max(16, min_T). `throughput`:
// cost of a share of a large batch (no rounding to whole waves of workgroups) instead of
// one launch on its own. Uses the context's measured per-block costs when the autotuner
// has calibrated them, else a static operation count.
bool pick_tile(ecc_context ctx, int R, int U, int ny, int nx, int batch, bool throughput, int min_T,
               TileChoice& best);
// Measures the per-block cost of every compiled block shape on the context's device
// (once per context; later calls return at once).
ecc_status calibrate_tiles(ecc_context ctx, hipStream_t st);
// Same choice for the tiled convolution (static operation count).
bool pick_tile_conv(ecc_context ctx, int R, int U, int ny, int nx, int batch, int min_T, TileChoice& best);
// Whether the direct (spatial) correlation (conv: convolution) is expected to beat the
// block path for a filter side S with U components on batch x ny x nx images.
bool direct_preferred(ecc_context ctx, bool conv, int S, int U, int ny, int nx, int batch);
// Block shape of the overlap-add ratio kernel for the plan's filter radius R (plans with
// component parity only): among the compiled shapes, the smallest transform work per
// output pixel, N^2 log2 N / T^2 with T = min(TV, N - 2R) >= 16. The normalised
// convolution takes it where the block convolution would use N = 128.
bool pick_tile_ratio(ecc_filter_plan plan, TileChoice& best);
// Block spectra of a plan for transform length N (cached in the plan): for correlation
// (F_k with its window corner at (0, 0)), convolution (offset x at (x - R) mod N, padded
// planes) or the symmetric correlation form (centred: offset x at x mod N); the _CONJ
// modes are those of conj(F_k) (the adjoint correlates with F_k itself).
// SPEC_RATIO: the float2 planes of the overlap-add ratio kernel (launch_ratio_spectra).
enum { SPEC_CORR = 0, SPEC_CONV = 1, SPEC_CENTRED = 2, SPEC_CORR_CONJ = 3, SPEC_CENTRED_CONJ = 4, SPEC_RATIO = 5 };
ecc_status get_tile_spectrum(ecc_filter_plan plan, int N, hipStream_t st, const Spectrum** out, int mode = SPEC_CORR);
// The cached block spectra of get_tile_spectrum, or NULL if they have not been built
// (builds nothing and allocates nothing).
const Spectrum* find_tile_spectrum(ecc_filter_plan plan, int N, int mode);
// rotation plans: F_k(-x) = (-1)^k F_k(x), components k = 0 .. U - 1
bool rotation_parity(ecc_filter_plan plan);
// Per-pixel angle description of a plan's field argument.
Field make_field(ecc_filter_plan plan, const float* f, long long plane, int ld, double mul_sign);
// Any forward operator call (validated arguments) on stream st.
ecc_status forward_impl(ecc_context ctx, ecc_op op, ecc_filter_plan plan, int batch, int ny, int nx,
                        const float* signal, int ld_signal, const float* field, int ld_field,
                        float* out, int ld_out, hipStream_t st, void* saved);
// Common checks of a call's images; `joint`: the call takes rotation-and-scale plans (and
// only those), else it refuses them.
ecc_status validate_images(ecc_filter_plan plan, int batch, int ny, int nx, bool joint = false);
bool overlaps(const void* a, size_t na, const void* b, size_t nb);
// Frees the volume plans still alive in a context that is being destroyed.
void destroy_volume_plans(ecc_context ctx);

}  // namespace ecc
