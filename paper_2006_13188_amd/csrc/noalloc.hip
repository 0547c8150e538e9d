// Rotation matching that allocates nothing: the component stack of the block strategy
// goes through a fixed device array of this library instead of the context workspace,
// one band of block rows at a time (stack kernel, then the angle search of the band).
//
// The array is a file-scope __device__ object: every GPU the library runs on holds its
// own copy until the process ends. In host code its name is only a host-side stand-in,
// so its device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and only that address is handed to kernels.
#include <mutex>

#include "api_common.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
ecc_status scratch_for(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return ecc::fail(ECC_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return ecc::fail(ECC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return ECC_OK;
}

}  // namespace

extern "C" {

ecc_status ecc_match_rotations_noalloc(ecc_context ctx, ecc_filter_plan plan, int ny, int nx, const float* signal,
                                       int ld, int n_angles, float* best_score, int* best_index, int ld_out,
                                       ecc_precision prec, void* stream) {
  using namespace ecc;
  ECC_REQ(ctx && plan, "NULL context or plan");
  ECC_REQ(plan->ctx == ctx, "plan belongs to another context");
  ECC_REQ(plan->group == ECC_GROUP_ROTATION, "matching needs a rotation plan");
  ECC_REQ(signal && best_score && best_index, "NULL pointer");
  ECC_REQ(prec == ECC_PREC_FP32 || prec == ECC_PREC_MFMA_FP16_HILO || prec == ECC_PREC_MFMA_BF16_HILO,
          "unknown precision");
  ECC_TRY(validate_images(plan, 1, ny, nx));
  ECC_REQ(ld >= nx && ld_out >= nx, "row strides must be >= nx");
  ECC_REQ(n_angles >= 2 * plan->K + 1 && n_angles <= 64, "need 2K+1 <= n_angles <= 64");
  if (ctx->autotune && !ctx->tile_calibrated)
    return fail(ECC_ERR_UNSUPPORTED,
                "the autotuner has not calibrated this context yet (its timing runs allocate): make one "
                "allocating call first");
  const int R = plan->R, U = plan->U;
  TileChoice tc;
  const bool tiled = ctx->strategy != ECC_STRATEGY_TWO_PASS &&
                     pick_tile(ctx, R, U, ny, nx, 1, false, ctx->strategy == ECC_STRATEGY_AUTO ? 2 * R : 16, tc);
  if (!tiled)
    return fail(ECC_ERR_UNSUPPORTED,
                "no block shape for this filter radius under the context's strategy (the whole-image form "
                "needs the context workspace)");
  const bool sym = tile_symmetric(tc.N, tc.TV) && rotation_parity(plan);
  const Spectrum* sp = find_tile_spectrum(plan, tc.N, sym ? SPEC_CENTRED : SPEC_CORR);
  if (!sp || plan->match_tab_A != n_angles)
    return fail(ECC_ERR_UNSUPPORTED,
                "the plan's block spectra or angle table for this image size and angle count do not exist yet: "
                "run ecc_match_rotations once with the same plan, size and n_angles first");
  // a band of b block rows takes U planes of stack_pitch(b T nx) complex values
  const int nby = (ny + tc.T - 1) / tc.T;
  auto band_bytes = [&](int b) {
    return (size_t)U * (size_t)stack_pitch((long long)std::min(ny, b * tc.T) * nx) * sizeof(float2);
  };
  if (band_bytes(1) > kScratchBytes)
    return fail(ECC_ERR_INVALID_ARGUMENT,
                "one block row of the component stack (" + std::to_string(band_bytes(1)) + " bytes) exceeds the " +
                    std::to_string(kScratchBytes) + "-byte scratch array: use ecc_match_rotations");
  DeviceGuard dg(ctx->device);
  hipStream_t st = S(stream);
  void* scr = nullptr;
  ECC_TRY(scratch_for(ctx->device, &scr));
  float* stack = static_cast<float*>(scr);
  int band = 1;   // block rows per band: the most that fit
  while (band < nby && band_bytes(band + 1) <= kScratchBytes) ++band;
  const int pc = prec == ECC_PREC_FP32 ? 0 : (prec == ECC_PREC_MFMA_FP16_HILO ? 1 : 2);
  const float scale = 1.0f / ((float)tc.N * (float)tc.N);
  for (int by0 = 0; by0 < nby; by0 += band) {
    const int by1 = std::min(nby, by0 + band);
    const int y0 = by0 * tc.T, rows = std::min(ny, by1 * tc.T) - y0;
    ECC_HIP(launch_tile_stack(st, tc.N, tc.TV, signal, ld, ny, nx, R, tc.T, U, scale, sp->buf.as<cx<float>>(),
                              stack, sym, by0, by1));
    ECC_HIP(launch_match_angles(st, pc, stack, U, (long long)rows * nx, n_angles, plan->match_tab.as<float>(),
                                best_score + (long long)y0 * ld_out, best_index + (long long)y0 * ld_out, ld_out,
                                nx));
  }
  return ECC_OK;
}

}  // extern "C"
