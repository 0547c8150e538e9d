// Internal host-side state of libecc: contexts, transforms, filter plans.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/ecc.h"
#include "kernels.hpp"

struct ecc_context_s;
struct ecc_volume_plan_s;

namespace ecc {

struct Transform {
  FftDesc desc{};
  std::vector<int> rad;
  void* tw32 = nullptr;   // cx<float>[twsize]
  void* tw64 = nullptr;   // cx<double>[twsize]
  int fR0 = 0, fR1 = 0, fR2 = 0;   // compiled three-pass schedule (fR0 = 0 if none)
  void* fx_tw32 = nullptr;         // its pass-1 and pass-2 twiddle tables
  ~Transform();
  const cx<float>* f() const { return static_cast<const cx<float>*>(tw32); }
  const cx<double>* d() const { return static_cast<const cx<double>*>(tw64); }
  const cx<float>* fx() const { return static_cast<const cx<float>*>(fx_tw32); }
};

hipError_t get_transform(ecc_context_s* ctx, int P, const Transform** out);
bool is_smooth7(int n);
int next_smooth7(int n);
std::vector<int> choose_radices(int P);
int max_butterflies(const Transform& t);
RowCfg row_config(const Transform& t, int span, size_t elem, int max_threads = 256);
ColCfg col_config(const Transform& t, int want_lgB, size_t elem, int nthr);

// Device buffer owned by the library.
struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    if (p) {
      (void)hipDeviceSynchronize();   // queued kernels may still use the old buffer
      hipError_t e = hipFree(p);
      p = nullptr;
      n = 0;
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) n = bytes;
    return e;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

}  // namespace ecc

struct ecc_context_s {
  int device = 0;
  std::mutex mu;
  std::map<int, std::unique_ptr<ecc::Transform>> transforms;
  ecc::DevBuf ws;           // per-call workspace (grown on demand)
  hipStream_t ws_stream = nullptr;   // stream of the last call that used ws
  hipEvent_t ws_event = nullptr;     // recorded on it after that call's last kernel
  ecc::DevBuf angle_tab;    // cos/sin tables for matching
  int angle_tab_n = 0;
  int autotune = 0;
  ecc_strategy strategy = ECC_STRATEGY_AUTO;
  std::map<std::string, int> tuned;   // shape key -> chosen FFT size
  std::vector<hipEvent_t> stage_events;   // measurement hook (see ecc_set_stage_events)
  std::set<ecc_filter_plan_s*> plans;     // live plans made from this context
  std::set<ecc_volume_plan_s*> vplans;    // live volume plans made from this context
  // measured cost of one full wave of blocks of each tiled shape (N, TV): t = a + b U (ms)
  struct TileCost {
    double a = 0, b = 0;
  };
  std::map<std::pair<int, int>, TileCost> tile_cost;
  bool tile_calibrated = false;
  int num_cus = 0;
};

struct Spectrum {
  int Py = 0, Px = 0, ld = 0, full = 0;
  ecc::DevBuf buf;   // U planes of Py x ld complex64
};

struct ecc_filter_plan_s {
  ecc_context ctx = nullptr;
  int device = 0;
  ecc_group group = ECC_GROUP_ROTATION;
  int S = 0, R = 0, K = 0, U = 0, M = 0;
  ecc::DevBuf comps64;   // U x S x S complex128
  ecc::DevBuf comps32;   // U x S x S complex64
  std::vector<float> weights;
  ecc::DevBuf d_weights;
  std::vector<float> parity;   // F_k(-x) = parity_k F_k(x), or empty
  ecc::DevBuf d_parity;
  int symmetric = 1;
  // per-pixel angle: alpha = field_mul * (log_mode ? ln f : f)
  double field_mul = 1.0;
  int log_mode = 0;
  int sig_norm = 0;   // divide the signal by field^2 (scale group)
  int joint_n = 0;    // joint rotation and scale plans: log-radial modes n (odd), else 0
  double joint_om1 = 0.0;   // omega_1 = 2 pi / L
  std::mutex mu;
  std::map<std::pair<int, int>, std::unique_ptr<Spectrum>> spectra;
  std::map<int, std::unique_ptr<Spectrum>> tile_spectra;   // N -> U planes of N x N
  ecc::DevBuf match_tab;       // angle-search matrix [64][64] for match_tab_A angles
  int match_tab_A = 0;
};
