// Pattern detection by extended convolution (section "Application to Pattern Detection"):
// the gradient signal and angle field of an image (eq. signal, eq. theta), the consensus
// filter of a pattern by voting (eq. opt_filt), and peak picking on the response.
#include <algorithm>
#include <hipcub/hipcub.hpp>

#include "kcommon.hpp"

namespace ecc {

namespace {

// H = |grad I|, theta = atan2(I_y, I_x): central differences inside, one-sided on the first
// and last row / column (x = column, y = row); one thread per pixel.
__global__ void __launch_bounds__(256) k_gradient_field(const float* __restrict__ I, long long planeI, int ldI,
                                                        int ny, int nx, float* __restrict__ H,
                                                        float* __restrict__ theta, long long planeO, int ldO) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, img = blockIdx.z;
  if (x >= nx) return;
  const float* row = I + (long long)img * planeI + (long long)y * ldI;
  float gx, gy;
  if (x == 0) gx = row[1] - row[0];
  else if (x == nx - 1) gx = row[nx - 1] - row[nx - 2];
  else gx = 0.5f * (row[x + 1] - row[x - 1]);
  if (y == 0) gy = row[ldI + x] - row[x];
  else if (y == ny - 1) gy = row[x] - row[x - ldI];
  else gy = 0.5f * (row[x + ldI] - row[x - ldI]);
  const long long o = (long long)img * planeO + (long long)y * ldO + x;
  H[o] = sqrtf(gx * gx + gy * gy);
  theta[o] = atan2f(gy, gx);
}

// Per pattern pixel (float64): the vote weight |grad P| and the vote position
// R_{-theta} (c - x) in window coordinates (column, row); weight 0 outside the disk.
__global__ void __launch_bounds__(256) k_vote_sources(const float* __restrict__ P, int S, double* __restrict__ src) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= S * S) return;
  const int i = k / S, j = k - i * S, R = (S - 1) / 2;
  auto at = [&](int r, int c) { return (double)P[r * S + c]; };
  const double gx = j == 0 ? at(i, 1) - at(i, 0) : j == S - 1 ? at(i, S - 1) - at(i, S - 2)
                                                              : 0.5 * (at(i, j + 1) - at(i, j - 1));
  const double gy = i == 0 ? at(1, j) - at(0, j) : i == S - 1 ? at(S - 1, j) - at(S - 2, j)
                                                              : 0.5 * (at(i + 1, j) - at(i - 1, j));
  const double h = sqrt(gx * gx + gy * gy);
  const int qx = j - R, qy = i - R;
  double w = 0.0, fx = 0.0, fy = 0.0;
  if (qx * qx + qy * qy <= R * R && h != 0.0) {
    const double c = gx / h, s = gy / h;   // cos and sin of the gradient angle
    const double vx = -qx, vy = -qy;       // c - x
    w = h;
    fx = c * vx + s * vy + R;
    fy = -s * vx + c * vy + R;
  }
  src[3 * k] = w;
  src[3 * k + 1] = fx;
  src[3 * k + 2] = fy;
}

// Filter bin (r, c) = sum over the sources, in raster order, of w max(0, 1 - |fx - c|)
// max(0, 1 - |fy - r|): the bilinear split of every vote, gathered per bin (float64, a
// fixed order, no atomics); rounded to float32 once.
__global__ void __launch_bounds__(256) k_vote_gather(const double* __restrict__ src, int S, float* __restrict__ F) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= S * S) return;
  const int r = k / S, c = k - r * S;
  double acc = 0.0;
  for (int q = 0; q < S * S; ++q) {
    const double w = src[3 * q];
    if (w == 0.0) continue;
    const double ax = 1.0 - fabs(src[3 * q + 1] - c), ay = 1.0 - fabs(src[3 * q + 2] - r);
    if (ax > 0.0 && ay > 0.0) acc += w * ay * ax;
  }
  F[k] = (float)acc;
}

// order-preserving map of a float to an unsigned integer
__device__ __forceinline__ unsigned int ordered(float v) {
  const unsigned int u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unordered(unsigned int o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

__global__ void __launch_bounds__(256) k_fill_u64(unsigned long long* __restrict__ a, long long n,
                                                  unsigned int* __restrict__ counter, unsigned int* __restrict__ mx) {
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k < n) a[k] = 0ull;
  if (k == 0) {
    *counter = 0u;
    *mx = 0u;   // below every ordered value
  }
}

// largest response (ordered encoding; max is independent of the order of the updates)
// (each workgroup reduces a stripe of rows in registers, then through LDS, and adds one
// atomic maximum: a few hundred atomics on the one word instead of one per wave)
__global__ void __launch_bounds__(256) k_max_response(const float* __restrict__ D, int ld, int ny, int nx,
                                                      unsigned int* __restrict__ mx) {
  __shared__ unsigned int wmax[4];
  unsigned int v = 0u;
  for (int y = blockIdx.x; y < ny; y += gridDim.x)
    for (int x = threadIdx.x; x < nx; x += 256) v = max(v, ordered(D[(long long)y * ld + x]));
  for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned int)__shfl_xor((int)v, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    v = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
    if (v) atomicMax(mx, v);
  }
}

// A pixel is a peak if its response is >= the threshold (thr, or rel times the largest
// response when rel > 0), no response in the (2r+1)^2 window is larger, and no earlier
// pixel (raster order) in it is equal. Peaks go to a list as 64-bit keys: ordered value in
// the high word, ~index in the low word (so a descending sort lists larger values first and
// equal values by increasing index).
__global__ void __launch_bounds__(256) k_mark_peaks(const float* __restrict__ D, int ld, int ny, int nx, int rad,
                                                    float thr, float rel, const unsigned int* __restrict__ mx,
                                                    unsigned long long* __restrict__ keys, unsigned int cap,
                                                    unsigned int* __restrict__ counter) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  if (x >= nx) return;
  const float v = D[(long long)y * ld + x];
  const float t = rel > 0.f ? rel * unordered(*mx) : thr;
  if (!(v >= t)) return;
  const int y0 = max(0, y - rad), y1 = min(ny - 1, y + rad), x0 = max(0, x - rad), x1 = min(nx - 1, x + rad);
  for (int yy = y0; yy <= y1; ++yy)
    for (int xx = x0; xx <= x1; ++xx) {
      const float w = D[(long long)yy * ld + xx];
      if (w > v || (w == v && (yy < y || (yy == y && xx < x)))) return;
    }
  const unsigned int slot = atomicAdd(counter, 1u);
  if (slot < cap) {
    const unsigned int idx = (unsigned int)y * (unsigned int)nx + (unsigned int)x;
    keys[slot] = ((unsigned long long)ordered(v) << 32) | (unsigned long long)(~idx);
  }
}

// The same test with the window read from LDS: a workgroup covers a tile of kPkTx x kPkTy
// pixels and stages its (kPkTx + 2 rad) x (kPkTy + 2 rad) neighbourhood once (positions
// outside the image hold NaN, which no comparison selects, as the image border clips the
// window in the form above). The window maximum comes from two one-dimensional passes
// (rows, then columns; fmaxf skips NaN), so every thread does the same 2 (2 rad + 1)
// steps; only a pixel equal to its window maximum then scans the window for an earlier
// equal value. Launched for rad <= kPkMaxRad.
constexpr int kPkTx = 64, kPkTy = 4, kPkMaxRad = 32;

__global__ void __launch_bounds__(256) k_mark_peaks_tile(const float* __restrict__ D, int ld, int ny, int nx, int rad,
                                                         float thr, float rel, const unsigned int* __restrict__ mx,
                                                         unsigned long long* __restrict__ keys, unsigned int cap,
                                                         unsigned int* __restrict__ counter) {
  extern __shared__ float win[];
  const int W = kPkTx + 2 * rad, Hh = kPkTy + 2 * rad;
  float* rmax = win + W * Hh;   // Hh rows x kPkTx: maximum over each row's 2 rad + 1 window
  const int tx0 = blockIdx.x * kPkTx - rad, ty0 = blockIdx.y * kPkTy - rad;
  for (int e = threadIdx.x; e < W * Hh; e += 256) {
    const int yy = ty0 + e / W, xx = tx0 + e % W;
    win[e] = (yy >= 0 && yy < ny && xx >= 0 && xx < nx) ? D[(long long)yy * ld + xx] : __builtin_nanf("");
  }
  __syncthreads();
  for (int e = threadIdx.x; e < Hh * kPkTx; e += 256) {
    const int ry = e / kPkTx, cx_ = e % kPkTx;
    const float* wr = win + ry * W + cx_;
    float m = wr[0];
    for (int d = 1; d <= 2 * rad; ++d) m = fmaxf(m, wr[d]);
    rmax[e] = m;
  }
  __syncthreads();
  const int lx = threadIdx.x % kPkTx, ly = threadIdx.x / kPkTx;
  const int x = blockIdx.x * kPkTx + lx, y = blockIdx.y * kPkTy + ly;
  if (x >= nx || y >= ny) return;
  const float v = win[(ly + rad) * W + lx + rad];
  const float t = rel > 0.f ? rel * unordered(*mx) : thr;
  if (!(v >= t)) return;
  float wm = rmax[ly * kPkTx + lx];
  for (int d = 1; d <= 2 * rad; ++d) wm = fmaxf(wm, rmax[(ly + d) * kPkTx + lx]);
  if (wm > v) return;
  // v is the window maximum: it is the peak unless an equal value comes earlier in raster order
  for (int dy = -rad; dy <= 0; ++dy) {
    const float* wr = win + (ly + rad + dy) * W + lx + rad;
    const int dx1 = dy < 0 ? rad : -1;
    for (int dx = -rad; dx <= dx1; ++dx)
      if (wr[dx] == v) return;
  }
  const unsigned int slot = atomicAdd(counter, 1u);
  if (slot < cap) {
    const unsigned int idx = (unsigned int)y * (unsigned int)nx + (unsigned int)x;
    keys[slot] = ((unsigned long long)ordered(v) << 32) | (unsigned long long)(~idx);
  }
}

__global__ void __launch_bounds__(256) k_emit_peaks(const unsigned long long* __restrict__ sorted, int nx, int max_peaks,
                                                    const unsigned int* __restrict__ counter, int* __restrict__ rows,
                                                    int* __restrict__ cols, float* __restrict__ vals,
                                                    int* __restrict__ count) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int n = (int)min((unsigned int)max_peaks, *counter);
  if (k == 0) *count = n;
  if (k >= n) return;
  const unsigned long long key = sorted[k];
  const unsigned int idx = ~(unsigned int)(key & 0xffffffffull);
  rows[k] = (int)(idx / (unsigned int)nx);
  cols[k] = (int)(idx % (unsigned int)nx);
  vals[k] = unordered((unsigned int)(key >> 32));
}

}  // namespace

hipError_t launch_gradient_field(hipStream_t s, int batch, int ny, int nx, const float* I, long long planeI, int ldI,
                                 float* H, float* theta, long long planeO, int ldO) {
  if (ny < 2 || nx < 2 || batch < 1 || ny > 65535 || batch > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gradient_field, dim3((unsigned)((nx + 255) / 256), (unsigned)ny, (unsigned)batch), dim3(256),
                     0, s, I, planeI, ldI, ny, nx, H, theta, planeO, ldO);
  return last();
}

size_t voting_scratch_bytes(int S) { return (size_t)S * S * 3 * sizeof(double); }

hipError_t launch_voting_filter(hipStream_t s, const float* P, int S, float* F, void* scratch) {
  if (S < 3 || S % 2 == 0) return hipErrorInvalidValue;
  double* src = static_cast<double*>(scratch);
  const unsigned g = (unsigned)((S * S + 255) / 256);
  hipLaunchKernelGGL(k_vote_sources, dim3(g), dim3(256), 0, s, P, S, src);
  hipError_t e = last();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vote_gather, dim3(g), dim3(256), 0, s, src, S, F);
  return last();
}

// peaks are more than `rad` apart in both directions: at most one per (rad+1)^2 cell
long long peak_capacity(int ny, int nx, int rad) {
  return (long long)((ny + rad) / (rad + 1)) * (long long)((nx + rad) / (rad + 1));
}

size_t peak_scratch_bytes(int ny, int nx, int rad) {
  const long long cap = peak_capacity(ny, nx, rad);
  size_t tmp = 0;
  (void)hipcub::DeviceRadixSort::SortKeysDescending(nullptr, tmp, (const unsigned long long*)nullptr,
                                                    (unsigned long long*)nullptr, (int)cap);
  return 256 + 2 * (size_t)cap * sizeof(unsigned long long) + ((tmp + 255) / 256) * 256;
}

hipError_t launch_find_peaks(hipStream_t s, const float* D, int ld, int ny, int nx, int rad, float thr, float rel,
                             int max_peaks, int* rows, int* cols, float* vals, int* count, void* scratch,
                             size_t scratch_bytes) {
  if (ny < 1 || nx < 1 || ny > 65535 || rad < 0 || max_peaks < 1) return hipErrorInvalidValue;
  const long long cap = peak_capacity(ny, nx, rad);
  if (cap > 0x7fffffffLL || scratch_bytes < peak_scratch_bytes(ny, nx, rad)) return hipErrorInvalidValue;
  char* base = static_cast<char*>(scratch);
  unsigned int* counter = reinterpret_cast<unsigned int*>(base);
  unsigned int* mx = counter + 1;
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(base + 256);
  unsigned long long* sorted = keys + cap;
  void* tmp = base + 256 + 2 * (size_t)cap * sizeof(unsigned long long);
  size_t tmp_bytes = scratch_bytes - (256 + 2 * (size_t)cap * sizeof(unsigned long long));
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, keys, cap, counter, mx);
  hipError_t e = last();
  if (e != hipSuccess) return e;
  if (rel > 0.f) {
    hipLaunchKernelGGL(k_max_response, dim3((unsigned)std::min(ny, 1024)), dim3(256), 0, s, D, ld, ny, nx, mx);
    if ((e = last()) != hipSuccess) return e;
  }
  if (rad <= kPkMaxRad) {
    const dim3 grid((unsigned)((nx + kPkTx - 1) / kPkTx), (unsigned)((ny + kPkTy - 1) / kPkTy));
    const size_t lds = sizeof(float) * (size_t)(kPkTy + 2 * rad) * (kPkTx + 2 * rad + kPkTx);
    hipLaunchKernelGGL(k_mark_peaks_tile, grid, dim3(256), lds, s, D, ld, ny, nx, rad, thr, rel, mx, keys,
                       (unsigned int)cap, counter);
  } else {
    const dim3 grid((unsigned)((nx + 255) / 256), (unsigned)ny);
    hipLaunchKernelGGL(k_mark_peaks, grid, dim3(256), 0, s, D, ld, ny, nx, rad, thr, rel, mx, keys,
                       (unsigned int)cap, counter);
  }
  if ((e = last()) != hipSuccess) return e;
  e = hipcub::DeviceRadixSort::SortKeysDescending(tmp, tmp_bytes, keys, sorted, (int)cap, 0, 64, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_emit_peaks, dim3((unsigned)((max_peaks + 255) / 256)), dim3(256), 0, s, sorted, nx, max_peaks,
                     counter, rows, cols, vals, count);
  return last();
}

}  // namespace ecc
