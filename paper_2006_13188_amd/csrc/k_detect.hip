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

// Adds `key`, for every lane with `take` set, to its workgroup's slots: one update of the
// workgroup's LDS counter per wave, slots in lane order after it. Every active lane of the
// wave must make the call. (A counter shared by the whole device would be one memory-side
// atomic per peak, serialised on one address: thousands of them took ~50 us at 1024^2.)
__device__ __forceinline__ void append_keys(bool take, unsigned long long key, unsigned long long* __restrict__ slots,
                                            unsigned int nslot, unsigned int* wcnt) {
  const unsigned long long m = __ballot(take);
  if (m == 0ull) return;
  const int lane = __lane_id();
  const int first = __ffsll((unsigned long long)m) - 1;
  unsigned int base = 0u;
  if (lane == first) base = atomicAdd(wcnt, (unsigned int)__popcll(m));
  base = (unsigned int)__shfl((int)base, first);
  if (take) {
    const unsigned int slot = base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
    if (slot < nslot) slots[slot] = key;
  }
}

// Zeroes the workgroup's slots past its last key (zero sorts below every peak's key). Every
// thread of the workgroup must make the call, after its last append.
__device__ __forceinline__ void zero_unused(unsigned long long* __restrict__ slots, unsigned int nslot,
                                            const unsigned int* wcnt) {
  __syncthreads();
  for (unsigned int i = min(*wcnt, nslot) + threadIdx.x; i < nslot; i += blockDim.x) slots[i] = 0ull;
}

// A pixel is a peak if its response is >= thr, no response in the (2r+1)^2 window is
// larger, and no earlier pixel (raster order) in it is equal. Peaks go to a list as 64-bit
// keys: ordered value in the high word, ~index in the low word (so a descending sort lists
// larger values first and equal values by increasing index), each workgroup's in its own
// slots (as many as peaks fit in its pixels: peaks are more than r apart in y or x), the
// unused ones set to zero so that they sort last. A relative threshold is
// applied after the sort: the largest response of the image is the value of its first peak
// (the first pixel holding the maximum is one), so the list is marked with thr = -inf and
// cut where the values fall below rel times the first.
__global__ void __launch_bounds__(256) k_mark_peaks(const float* __restrict__ D, int ld, int ny, int nx, int rad,
                                                    float thr, unsigned long long* __restrict__ keys, unsigned int spw) {
  __shared__ unsigned int wcnt;
  if (threadIdx.x == 0) wcnt = 0u;
  __syncthreads();
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  bool peak = false;
  float v = 0.f;
  if (x < nx) {
    v = D[(long long)y * ld + x];
    peak = v >= thr;
    const int y0 = max(0, y - rad), y1 = min(ny - 1, y + rad), x0 = max(0, x - rad), x1 = min(nx - 1, x + rad);
    for (int yy = y0; yy <= y1 && peak; ++yy)
      for (int xx = x0; xx <= x1; ++xx) {
        const float w = D[(long long)yy * ld + xx];
        if (w > v || (w == v && (yy < y || (yy == y && xx < x)))) {
          peak = false;
          break;
        }
      }
  }
  const unsigned int idx = (unsigned int)y * (unsigned int)nx + (unsigned int)x;
  unsigned long long* slots = keys + ((long long)blockIdx.y * gridDim.x + blockIdx.x) * spw;
  append_keys(peak, ((unsigned long long)ordered(v) << 32) | (unsigned long long)(~idx), slots, spw, &wcnt);
  zero_unused(slots, spw, &wcnt);
}

// The same test with the window read from LDS: a workgroup of 256 threads covers a tile of
// kPkTx x kPkTy pixels and stages its (kPkTx + 2 rad) x (kPkTy + 2 rad) neighbourhood once
// (positions outside the image hold NaN, which no comparison selects, as the image border
// clips the window in the form above). The window maxima come from two one-dimensional
// passes (rows, then columns; fmaxf skips NaN), the column pass split so that the same
// reads also give the maximum over the pixels before the centre in raster order (the rows
// above and the left part of the centre's row): a pixel is a peak iff that maximum is not
// equal to it and nothing in the window is larger, with no per-pixel scan (a scan that
// stops at the first earlier equal value makes each wave holding a local maximum wait on
// ~(rad + 1)(2 rad + 1) dependent LDS reads). A wave owns the 64 columns of a group of
// four rows (no LDS bank conflicts along a row), and a thread the four pixels of one
// column in it. Launched for rad <= kPkMaxRad.
constexpr int kPkTx = 64, kPkTy = 16, kPkMaxRad = 32;

__global__ void __launch_bounds__(256) k_mark_peaks_tile(const float* __restrict__ D, int ld, int ny, int nx, int rad,
                                                         float thr, unsigned long long* __restrict__ keys,
                                                         unsigned int spw) {
  extern __shared__ float win[];
  __shared__ unsigned int wcnt;
  if (threadIdx.x == 0) wcnt = 0u;
  const int W = kPkTx + 2 * rad, Hh = kPkTy + 2 * rad;
  float* rmax = win + W * Hh;   // Hh rows x kPkTx: maximum over each row's 2 rad + 1 window
  const int tx0 = blockIdx.x * kPkTx - rad, ty0 = blockIdx.y * kPkTy - rad;
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
#pragma unroll 4
  for (int r = g; r < Hh; r += 4) {
    const int yy = ty0 + r;
    const bool rin = yy >= 0 && yy < ny;
    const float* src = D + (long long)(rin ? yy : 0) * ld;
    for (int q = c; q < W; q += 64) {
      const int xx = tx0 + q;
      win[r * W + q] = (rin && xx >= 0 && xx < nx) ? src[xx] : __builtin_nanf("");
    }
  }
  __syncthreads();
  for (int r = g; r < Hh; r += 4) {
    const float* wr = win + r * W + c;
    float m = wr[0];
#pragma unroll 4
    for (int d = 1; d <= 2 * rad; ++d) m = fmaxf(m, wr[d]);
    rmax[r * kPkTx + c] = m;
  }
  __syncthreads();
  const int x = blockIdx.x * kPkTx + c;
#pragma unroll 1
  for (int j = 0; j < 4; ++j) {
    const int ly = 4 * g + j, y = blockIdx.y * kPkTy + ly;
    bool peak = false;
    float v = 0.f;
    if (x < nx && y < ny) {
      v = win[(ly + rad) * W + c + rad];
      // maxima over the window rows above the pixel (`up`), over the part of its own row
      // left of it (`left`): together the window's pixels before it in raster order, and
      // over the rest (its whole row and the rows below). NaN is the empty maximum (fmaxf
      // skips it and it equals nothing), so positions outside the image drop out.
      float up = __builtin_nanf(""), left = __builtin_nanf(""), rest = rmax[(ly + rad) * kPkTx + c];
#pragma unroll 4
      for (int d = 0; d < rad; ++d) {
        up = fmaxf(up, rmax[(ly + d) * kPkTx + c]);
        rest = fmaxf(rest, rmax[(ly + rad + 1 + d) * kPkTx + c]);
        left = fmaxf(left, win[(ly + rad) * W + c + d]);
      }
      // a peak: nothing in the window larger, nothing before it equal
      peak = v >= thr && !(fmaxf(up, rest) > v) && !(fmaxf(up, left) == v);
    }
    const unsigned int idx = (unsigned int)y * (unsigned int)nx + (unsigned int)x;
    append_keys(peak, ((unsigned long long)ordered(v) << 32) | (unsigned long long)(~idx),
                keys + ((long long)blockIdx.y * gridDim.x + blockIdx.x) * spw, spw, &wcnt);
  }
  zero_unused(keys + ((long long)blockIdx.y * gridDim.x + blockIdx.x) * spw, spw, &wcnt);
}

// Writes the first min(max_peaks, n) peaks of the sorted slots (n = the nonzero keys, a
// prefix); with rel > 0 only those whose value is >= rel times the first one's (a shorter
// prefix). Both lengths by binary search.
__global__ void __launch_bounds__(256) k_emit_peaks(const unsigned long long* __restrict__ sorted, unsigned int nslots,
                                                    int nx, int max_peaks, float rel, int* __restrict__ rows,
                                                    int* __restrict__ cols, float* __restrict__ vals,
                                                    int* __restrict__ count) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  unsigned int m = 0u;
  {
    unsigned int hi = nslots;   // keys at [0, m) nonzero, at [hi, nslots) zero
    while (m < hi) {
      const unsigned int mid = (m + hi) >> 1;
      if (sorted[mid] != 0ull) m = mid + 1u;
      else hi = mid;
    }
  }
  if (rel > 0.f && m > 0u) {
    const float t = rel * unordered((unsigned int)(sorted[0] >> 32));
    unsigned int lo = 0u, hi = m;   // values at [0, lo) are >= t, at [hi, m) below t
    while (lo < hi) {
      const unsigned int mid = (lo + hi) >> 1;
      if (unordered((unsigned int)(sorted[mid] >> 32)) >= t) lo = mid + 1u;
      else hi = mid;
    }
    m = lo;
  }
  const int n = (int)min((unsigned int)max_peaks, m);
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
// Workgroups of the marking kernel and the key slots of each (the most peaks its pixels
// can hold: peaks are more than rad apart in y or x, one per (rad + 1)^2 cell at most).
void peak_slots(int ny, int nx, int rad, long long* nwg, long long* spw) {
  const long long c = rad + 1;
  if (rad <= kPkMaxRad) {
    *nwg = (long long)((nx + kPkTx - 1) / kPkTx) * ((ny + kPkTy - 1) / kPkTy);
    *spw = ((kPkTx + c - 1) / c) * ((kPkTy + c - 1) / c);
  } else {
    *nwg = (long long)((nx + 255) / 256) * ny;
    *spw = (256 + c - 1) / c;
  }
}

size_t peak_scratch_bytes(int ny, int nx, int rad) {
  long long nwg = 0, spw = 0;
  peak_slots(ny, nx, rad, &nwg, &spw);
  const long long n = nwg * spw;
  size_t tmp = 0;
  (void)hipcub::DeviceRadixSort::SortKeysDescending(nullptr, tmp, (const unsigned long long*)nullptr,
                                                    (unsigned long long*)nullptr, (int)n);
  return 2 * (size_t)n * sizeof(unsigned long long) + ((tmp + 255) / 256) * 256;
}

hipError_t launch_find_peaks(hipStream_t s, const float* D, int ld, int ny, int nx, int rad, float thr, float rel,
                             int max_peaks, int* rows, int* cols, float* vals, int* count, void* scratch,
                             size_t scratch_bytes) {
  if (ny < 1 || nx < 1 || ny > 65535 || rad < 0 || max_peaks < 1) return hipErrorInvalidValue;
  long long nwg = 0, spw = 0;
  peak_slots(ny, nx, rad, &nwg, &spw);
  const long long n = nwg * spw;
  if (n > 0x7fffffffLL || scratch_bytes < peak_scratch_bytes(ny, nx, rad)) return hipErrorInvalidValue;
  unsigned long long* keys = static_cast<unsigned long long*>(scratch);
  unsigned long long* sorted = keys + n;
  void* tmp = sorted + n;
  size_t tmp_bytes = scratch_bytes - 2 * (size_t)n * sizeof(unsigned long long);
  hipError_t e = hipSuccess;
  const float mark_thr = rel > 0.f ? -INFINITY : thr;
  if (rad <= kPkMaxRad) {
    const dim3 grid((unsigned)((nx + kPkTx - 1) / kPkTx), (unsigned)((ny + kPkTy - 1) / kPkTy));
    const size_t lds = sizeof(float) * (size_t)(kPkTy + 2 * rad) * (kPkTx + 2 * rad + kPkTx);
    hipLaunchKernelGGL(k_mark_peaks_tile, grid, dim3(256), lds, s, D, ld, ny, nx, rad, mark_thr, keys,
                       (unsigned int)spw);
  } else {
    const dim3 grid((unsigned)((nx + 255) / 256), (unsigned)ny);
    hipLaunchKernelGGL(k_mark_peaks, grid, dim3(256), 0, s, D, ld, ny, nx, rad, mark_thr, keys, (unsigned int)spw);
  }
  if ((e = last()) != hipSuccess) return e;
  e = hipcub::DeviceRadixSort::SortKeysDescending(tmp, tmp_bytes, keys, sorted, (int)n, 0, 64, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_emit_peaks, dim3((unsigned)((max_peaks + 255) / 256)), dim3(256), 0, s, sorted,
                     (unsigned int)n, nx, max_peaks, rel, rows, cols, vals, count);
  return last();
}

}  // namespace ecc
