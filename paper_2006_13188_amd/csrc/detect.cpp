// C ABI of the pattern-detection steps (section "Application to Pattern Detection"):
// gradient signal and field, consensus filter by voting, peak picking.
#include "api_common.hpp"

namespace ecc {
hipError_t launch_gradient_field(hipStream_t s, int batch, int ny, int nx, const float* I, long long planeI, int ldI,
                                 float* H, float* theta, long long planeO, int ldO);
size_t voting_scratch_bytes(int S);
hipError_t launch_voting_filter(hipStream_t s, const float* P, int S, float* F, void* scratch);
size_t peak_scratch_bytes(int ny, int nx, int rad);
hipError_t launch_find_peaks(hipStream_t s, const float* D, int ld, int ny, int nx, int rad, float thr, float rel,
                             int max_peaks, int* rows, int* cols, float* vals, int* count, void* scratch,
                             size_t scratch_bytes);
}  // namespace ecc

using namespace ecc;

extern "C" {

ecc_status ecc_gradient_field(ecc_context ctx, int batch, int ny, int nx, const float* image, int ld_image,
                              float* magnitude, float* angle, int ld_out, void* stream) {
  ECC_REQ(ctx, "NULL context");
  ECC_REQ(image && magnitude && angle, "NULL image pointer");
  ECC_REQ(batch >= 1 && batch <= 65535, "batch must be in [1, 65535]");
  ECC_REQ(ny >= 2 && nx >= 2 && ny <= 4096 && nx <= 4096, "image sides must be in [2, 4096]");
  ECC_REQ(ld_image >= nx && ld_out >= nx, "row strides must be >= nx");
  const size_t bi = (size_t)batch * ny * ld_image * sizeof(float), bo = (size_t)batch * ny * ld_out * sizeof(float);
  ECC_REQ(!overlaps(magnitude, bo, image, bi) && !overlaps(angle, bo, image, bi) && !overlaps(magnitude, bo, angle, bo),
          "outputs alias each other or the image");
  DeviceGuard dg(ctx->device);
  ECC_HIP(launch_gradient_field(S(stream), batch, ny, nx, image, (long long)ny * ld_image, ld_image, magnitude, angle,
                                (long long)ny * ld_out, ld_out));
  return ECC_OK;
}

ecc_status ecc_voting_filter(ecc_context ctx, int Sz, const float* pattern, float* filter, void* stream) {
  ECC_REQ(ctx, "NULL context");
  ECC_REQ(pattern && filter, "NULL pointer");
  ECC_REQ(Sz >= 3 && Sz <= 255 && Sz % 2 == 1, "pattern side must be odd, 3..255");
  const size_t b = (size_t)Sz * Sz * sizeof(float);
  ECC_REQ(!overlaps(filter, b, pattern, b), "filter aliases the pattern");
  DeviceGuard dg(ctx->device);
  hipStream_t st = S(stream);
  WsUse wu(ctx, st);
  ECC_HIP(ctx->ws.ensure(voting_scratch_bytes(Sz)));
  ECC_HIP(launch_voting_filter(st, pattern, Sz, filter, ctx->ws.p));
  return ECC_OK;
}

ecc_status ecc_find_peaks(ecc_context ctx, int ny, int nx, const float* response, int ld, int radius,
                          float threshold, int relative, int max_peaks, int* rows, int* cols, float* values,
                          int* count, void* stream) {
  ECC_REQ(ctx, "NULL context");
  ECC_REQ(response && rows && cols && values && count, "NULL pointer");
  ECC_REQ(ny >= 1 && nx >= 1 && ny <= 4096 && nx <= 4096, "image sides must be in [1, 4096]");
  ECC_REQ(ld >= nx, "row stride must be >= nx");
  ECC_REQ(radius >= 0 && radius <= 255, "radius must be in [0, 255]");
  ECC_REQ(max_peaks >= 1 && max_peaks <= (1 << 24), "max_peaks must be in [1, 2^24]");
  ECC_REQ(!relative || (threshold > 0.f && threshold <= 1.f), "a relative threshold must be in (0, 1]");
  DeviceGuard dg(ctx->device);
  hipStream_t st = S(stream);
  WsUse wu(ctx, st);
  const size_t need = peak_scratch_bytes(ny, nx, radius);
  ECC_HIP(ctx->ws.ensure(need));
  ECC_HIP(launch_find_peaks(st, response, ld, ny, nx, radius, relative ? 0.f : threshold, relative ? threshold : 0.f,
                            max_peaks, rows, cols, values, count, ctx->ws.p, ctx->ws.n));
  return ECC_OK;
}

}  // extern "C"
