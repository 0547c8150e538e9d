// Normalised extended convolution (image-filtering section, eq. normalization): the ratio
// of the extended convolutions of two signals that share the field,
//   num = sum_c w_c Re((s1 e^{-i c alpha}) * F_c),   den = the same with s2,
// s1 = H wn, s2 = wn (wn = 1 / field^2 for the scale group, 1 for rotations), by
// overlap-add blocks: every workgroup takes the T x T source pixels of one block,
// transforms them zero-padded to N x N (N >= T + 2R) and scatters the N x N region they
// reach into a partial-sum buffer; a second kernel adds the overlapping regions in a fixed
// order and divides.
//
// Both signals go through one set of transforms. With m_c = s e^{-i c alpha} = u - i v
// (u = s cos c alpha, v = s sin c alpha) and F_c = a_c + i b_c (a_c, b_c real),
// Re(m_c * F_c) = u * a_c + v * b_c, and convolution with a real filter keeps real and
// imaginary parts apart, so with the packed sources
//   P_c = (s1 + i s2) cos(c alpha),  Q_c = (s1 + i s2) sin(c alpha)
// sum_c w_c (P_c * a_c + Q_c * b_c) = num + i den: two forward transforms per component,
// one accumulator, one inverse transform per block.
//
// The components have parity F_c(-x) = p_c F_c(x) (rotation: (-1)^c; scale: radial, +1),
// so the centred spectra of a_c and b_c are real (p_c = 1) or imaginary (p_c = -1); the
// plan stores w_c times their real or imaginary parts as one float2 plane per component,
// transposed ([column frequency][row frequency]) so that the lanes of a wave (consecutive
// row frequencies) read consecutive values.
//
// Pruning: the sources fill rows and columns [0, T) of the window; column transforms run
// only over those T columns, and every radix-8 butterfly of the first pass of a line reads
// only its inputs below T (at most ceil(T / M) of the eight).
#include "mfma_split.hpp"
#include "tile_common.hpp"

namespace ecc {

namespace {

// length-8 DFT with inputs 4..7 zero: even outputs are the 4-point DFT of x_0..x_3, odd
// outputs the 4-point DFT of x_r w^r (w = exp(DIR 2 pi i / 8))
template <int DIR>
__device__ __forceinline__ void dft8_lo4(cx<float>* x) {
  cx<float> e[4] = {x[0], x[1], x[2], x[3]};
  cx<float> o[4] = {x[0], twiddle_const<8, DIR, float>(x[1], 1), twiddle_const<8, DIR, float>(x[2], 2),
                    twiddle_const<8, DIR, float>(x[3], 3)};
  dft<4, DIR, float>(e);
  dft<4, DIR, float>(o);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    x[2 * j] = e[j];
    x[2 * j + 1] = o[j];
  }
}
template <int RMAX, int DIR>
__device__ __forceinline__ void dft8_pruned(cx<float>* x) {
  if constexpr (RMAX <= 4) dft8_lo4<DIR>(x);
  else dft<8, DIR, float>(x);
}

// ---- 16-point DFTs on the matrix cores (float16 or bfloat16 hi + lo operands). For 16
// lines of one pass-1 butterfly at a time (a "tile", one wave): Y = X D with
// D[r][k] = exp(-2 pi i r k / 16), computed as Y^T = D^T X^T, so that lane l holds line
// l % 16 with elements r = 4 (l / 16) + j as its operand and gets back the same line with
// frequencies k = 4 (l / 16) + j. Complex products as real ones:
// Re Y = Re D Re X - Im D Im X, Im Y = Re D Im X + Im D Re X, each with hi/lo operands.
struct Cos16 {
  float c[16], s[16];
};
constexpr Cos16 make_cos16() {
  Cos16 t{};
  for (int m = 0; m < 16; ++m) {
    t.c[m] = (float)cos_turn(m, 16);
    t.s[m] = (float)sin_turn(m, 16);
  }
  return t;
}
__constant__ Cos16 kCos16 = make_cos16();

template <bool BF16>
struct D16Ops {
  typename Split<BF16>::T rh, rl, ih, il, nih, nil;   // Re D, Im D, -Im D (A operands, D^T)
};
template <bool BF16>
__device__ __forceinline__ D16Ops<BF16> make_d16(int lane) {
  const int lr = lane & 15, lq = lane >> 4;
  float re[4], im[4], nim[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int m = ((4 * lq + j) * lr) & 15;   // A[k = lr][r = 4 lq + j] = D[r][k]
    re[j] = kCos16.c[m];
    im[j] = -kCos16.s[m];
    nim[j] = kCos16.s[m];
  }
  D16Ops<BF16> d;
  Split<BF16>::split(re, d.rh, d.rl);
  Split<BF16>::split(im, d.ih, d.il);
  Split<BF16>::split(nim, d.nih, d.nil);
  return d;
}
// x: this lane's four (twiddled) elements of its line; y: its four outputs. float16
// operands are scaled per tile by a power of two so that the largest magnitude lies in
// [2^10, 2^11) (every lane of the wave takes part in the reduction).
template <bool BF16>
__device__ __forceinline__ void dft16_tile(const cx<float>* x, cx<float>* y, const D16Ops<BF16>& d) {
  using SP = Split<BF16>;
  float f = 1.f, inv = 1.f;
  if constexpr (!BF16) {
    float mx = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) mx = fmaxf(mx, fmaxf(fabsf(x[j].re), fabsf(x[j].im)));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    int ex = 0;
    (void)frexpf(mx, &ex);
    if (mx > 0.f) {
      f = ldexpf(1.f, 11 - ex);
      inv = ldexpf(1.f, ex - 11);
    }
  }
  float xr[4], xi[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    xr[j] = x[j].re * f;
    xi[j] = x[j].im * f;
  }
  typename SP::T xrh, xrl, xih, xil;
  SP::split(xr, xrh, xrl);
  SP::split(xi, xih, xil);
  f4_t yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
  yr = SP::mma(d.rh, xrh, yr);
  yr = SP::mma(d.rh, xrl, yr);
  yr = SP::mma(d.rl, xrh, yr);
  yr = SP::mma(d.nih, xih, yr);
  yr = SP::mma(d.nih, xil, yr);
  yr = SP::mma(d.nil, xih, yr);
  yi = SP::mma(d.rh, xih, yi);
  yi = SP::mma(d.rh, xil, yi);
  yi = SP::mma(d.rl, xih, yi);
  yi = SP::mma(d.ih, xrh, yi);
  yi = SP::mma(d.ih, xrl, yi);
  yi = SP::mma(d.il, xrh, yi);
#pragma unroll
  for (int j = 0; j < 4; ++j) y[j] = mk(yr[j] * inv, yi[j] * inv);
}

template <int N>
__shared__ cx<float> ratio_img_lds[N * (N + 1)];
// the sources' signal values, [pixel of the item][thread], and the phase step of each
// thread's first source pixel (kept out of the registers)
template <int NT, int NV>
__shared__ float ratio_h_lds[NV * NT];
template <int NT>
__shared__ cx<float> ratio_e1_lds[NT];

template <int N, int TV, int NT, int PREC, bool PLAIN>
__device__ __forceinline__ void ratio_block(const TileRatioArgs& a, int img, int tile, int blk, cx<float>* A) {
  constexpr int M = N / 8, P = N + 1, LS = NT / 8;
  constexpr int RMAX = (TV + M - 1) / M;        // pass-0 inputs that can lie below T
  constexpr int NQ0 = (TV * M + NT - 1) / NT;   // column pass-0 items (columns < TV)
  constexpr int NQR = (N * M + NT - 1) / NT;    // row pass-0 items (all N rows)
  constexpr int NI = (N + LS - 1) / LS;         // pass-1 lines over N lines
  constexpr int NIT = (TV + LS - 1) / LS;       // pass-1 lines over the source columns
  static_assert(RMAX <= 8, "source block wider than the window");
  // PREC 0: float32 radix-16 passes on the vector units; 1 / 2: the radix-16 passes of the
  // forward transforms (column pass 1, row pass 1 with the product) on the matrix cores,
  // float16 / bfloat16 hi + lo operands (tiles: 16 lines of one butterfly per wave)
  constexpr bool MF = PREC != 0;
  static_assert(!MF || (N == 128 && NT == 1024), "matrix-core passes: 128-point blocks, 16 waves");
  // PLAIN: one signal, y = Re sum_c w_c (m_c * F_c) with m_c = s1 e^{-i c alpha}: one
  // forward transform of the complex m_c per component, times the complex spectrum
  // F_c = a_c + i b_c (rho_a + i rho_b, or i rho_a - rho_b for odd parity)
  static_assert(!PLAIN || !MF, "the plain convolution runs on the vector units");
  constexpr int NPART = PLAIN ? 1 : 2;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int mlr = lane & 15, mlq = lane >> 4;
  const int mbq = wv & 7;   // the pass-1 butterfly of every tile of this wave
  const int t = threadIdx.x, l = t % LS;
  const int bq = (NT % 64 == 0 && LS % 64 == 0) ? __builtin_amdgcn_readfirstlane(t / LS) : t / LS;
  const int T = a.T;
  const int y0 = (tile / a.tx) * T, x0 = (tile % a.tx) * T;
  const TileTwiddles<N>& tt = tile_twiddles<N>();
  cx<float> tw[M];
  if constexpr (!MF) {
#pragma unroll
    for (int r = 0; r < M; ++r) tw[r] = mk(tt.re[bq][r], tt.im[bq][r]);
  }
  // matrix-core tiles: the pass-1 twiddles of this lane's elements r = 4 mlq + j, and D
  cx<float> twm[4];
  D16Ops<PREC == 2> d16;
  if constexpr (MF) {
#pragma unroll
    for (int j = 0; j < 4; ++j) twm[j] = mk(tt.re[mbq][4 * mlq + j], tt.im[mbq][4 * mlq + j]);
    d16 = make_d16<PREC == 2>(lane);
  }

  // ---- sources of this thread's column pass-0 items: h = H (0 outside), z = wn e^{i c alpha}
  // for the current component c (from c = 0), advanced by e1 = e^{i alpha}
  const float* Hb = a.H + (long long)img * a.planeH;
  float* hs = ratio_h_lds<NT, NQ0 * RMAX>;   // hs[(s RMAX + r) NT + t]
  cx<float> z[NQ0][RMAX], e1[NQ0][RMAX];
#pragma unroll
  for (int s = 0; s < NQ0; ++s) {
    const int q = t + s * NT;
    const int v = q % TV, b = q / TV;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      const int i = b + M * r;
      const int gy = y0 + i, gx = x0 + v;
      float hv = 0.f;
      z[s][r] = mk(0.f, 0.f);
      e1[s][r] = mk(0.f, 0.f);
      if (b < M && v < T && i < T && gy < a.ny && gx < a.nx) {
        const float fv = a.fld.ptr[(long long)img * a.fld.plane + (long long)gy * a.fld.ld + gx];
        float sn, cs;
        if (a.fld.log_mode) {
          double dsn, dcs;
          sincos(field_angle(a.fld, fv), &dsn, &dcs);
          sn = (float)dsn;
          cs = (float)dcs;
        } else {
          sincosf((float)a.fld.mul * fv + (float)a.fld.add, &sn, &cs);
        }
        e1[s][r] = mk(cs, sn);
        if (s == 0 && r == 0) ratio_e1_lds<NT>[t] = e1[0][0];   // read back only by this thread
        z[s][r] = mk(a.sig_norm ? 1.f / (fv * fv) : 1.f, 0.f);
        hv = Hb[(long long)gy * a.ldH + gx];
      }
      hs[(s * RMAX + r) * NT + t] = hv;   // read back only by this thread
    }
  }
  // accumulated spectrum bins of this thread: [line item][element] (vector units) or
  // [tile][j] (matrix cores: tile i is row group 2 i + wv / 8, bins (u, mbq + 8 (4 mlq + j)))
  constexpr int ZA = MF ? 4 : NI, ZB = MF ? 4 : M;
  cx<float> Z[ZA][ZB];
#pragma unroll
  for (int i = 0; i < ZA; ++i)
#pragma unroll
    for (int r = 0; r < ZB; ++r) Z[i][r] = mk(0.f, 0.f);

  // filter spectra through buffer loads: the lane offset u (consecutive lanes, one
  // register) plus a wave-uniform offset per element, so the addresses take no registers
  const __amdgpu_buffer_rsrc_t fsrc =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.Fs, (short)0, a.U * N * N * (int)sizeof(float2), 0x00020000);
  __syncthreads();   // the LDS image may still be in use by the previous block
  for (int c = 0; c < a.U; ++c) {
    const bool odd = a.par[c] < 0.f;   // spectra imaginary
#pragma unroll 1
    for (int part = 0; part < NPART; ++part) {   // P (cosine, with a_c), then Q (sine, with b_c)

      // ---- column pass 0 (radix 8, inputs below T only), straight from the sources
#pragma unroll
      for (int s = 0; s < NQ0; ++s) {
        const int q = t + s * NT;
        const int v = q % TV, b = q / TV;
        if (b < M && v < T) {
          cx<float> x[8];
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            if (r < RMAX) {
              if constexpr (PLAIN) {
                const float hv = hs[(s * RMAX + r) * NT + t];
                x[r] = mk(hv * z[s][r].re, -hv * z[s][r].im);
              } else {
                const float f = part ? z[s][r].im : z[s][r].re;
                x[r] = mk(hs[(s * RMAX + r) * NT + t] * f, f);
              }
            } else {
              x[r] = mk(0.f, 0.f);
            }
          }
          dft8_pruned<RMAX, -1>(x);
#pragma unroll
          for (int r = 0; r < 8; ++r) A[(8 * b + r) * P + v] = x[r];
        }
      }
      __syncthreads();
      // ---- column pass 1 over the T source columns
      if constexpr (MF) {
        // tiles (column group cg, butterfly mbq), in place: a lane reads elements
        // 4 mlq + j of its column and writes frequencies 4 mlq + j of the same column
        const int ncg = (T + 15) >> 4;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int cg = (wv >> 3) + 2 * i;
          if (cg < ncg) {
            const int v = 16 * cg + mlr;
            cx<float> x[4], y[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
              x[j] = v < T ? cmulc(A[(mbq + 8 * (4 * mlq + j)) * P + v], twm[j]) : mk(0.f, 0.f);
            dft16_tile<PREC == 2>(x, y, d16);
            if (v < T) {
#pragma unroll
              for (int j = 0; j < 4; ++j) A[(mbq + 8 * (4 * mlq + j)) * P + v] = y[j];
            }
          }
        }
      } else {
        pass1_inplace<N, -1, false, NIT, NT>(A, tw, bq, l, T, N);
      }
      __syncthreads();
      // ---- row pass 0 (radix 8, columns below T only), in NG groups of rows: a group's
      // outputs overwrite only its own rows, so the next group's inputs can be read right
      // after them, and only one group's values are held at a time
      {
        constexpr int NG = NQR % 2 == 0 ? 2 : 1, RG = N / NG, NQG = (RG * M + NT - 1) / NT;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          cx<float> xv[NQG][8];
#pragma unroll
          for (int s = 0; s < NQG; ++s) {
            const int q = t + s * NT;
            const int row = g * RG + q % RG, b = q / RG;
            if (b < M) {
#pragma unroll
              for (int r = 0; r < 8; ++r) {
                const int col = b + M * r;
                xv[s][r] = (r < RMAX && col < T) ? A[row * P + col] : mk(0.f, 0.f);
              }
            }
          }
          __syncthreads();
#pragma unroll
          for (int s = 0; s < NQG; ++s) {
            const int q = t + s * NT;
            const int row = g * RG + q % RG, b = q / RG;
            if (b < M) {
              dft8_pruned<RMAX, -1>(xv[s]);
#pragma unroll
              for (int r = 0; r < 8; ++r) A[row * P + 8 * b + r] = xv[s][r];
            }
          }
        }
      }
      __syncthreads();
      // ---- row pass 1 and the product with the (real or imaginary) filter spectrum
      if constexpr (MF) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int u = 16 * ((wv >> 3) + 2 * i) + mlr;
          cx<float> x[4], y[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) x[j] = cmulc(A[u * P + mbq + 8 * (4 * mlq + j)], twm[j]);
          dft16_tile<PREC == 2>(x, y, d16);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int vv = mbq + 8 * (4 * mlq + j);
            const float rho = __builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(
                           fsrc, (vv * N + u) * (int)sizeof(float2),
                           (c * N * N) * (int)sizeof(float2) + part * (int)sizeof(float), 0));
            if (odd) {
              Z[i][j].re -= y[j].im * rho;
              Z[i][j].im += y[j].re * rho;
            } else {
              Z[i][j].re += y[j].re * rho;
              Z[i][j].im += y[j].im * rho;
            }
          }
        }
      } else {
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int u = l + LS * i;
        if (N % LS == 0 || u < N) {
          cx<float> x[M];
#pragma unroll
          for (int r = 0; r < M; ++r) x[r] = A[u * P + bq + 8 * r];
#pragma unroll
          for (int r = 1; r < M; ++r) x[r] = cmulc(x[r], tw[r]);
          dft<M, -1, float>(x);
#pragma unroll
          for (int r = 0; r < M; ++r) {
            if constexpr (PLAIN) {
              const int so = ((c * N + bq + 8 * r) * N) * (int)sizeof(float2);
              const float ra = __builtin_bit_cast(
                  float, __builtin_amdgcn_raw_buffer_load_b32(fsrc, u * (int)sizeof(float2), so, 0));
              const float rb = __builtin_bit_cast(
                  float, __builtin_amdgcn_raw_buffer_load_b32(fsrc, u * (int)sizeof(float2), so + 4, 0));
              const cx<float> F = odd ? mk(-rb, ra) : mk(ra, rb);
              Z[i][r].re += x[r].re * F.re - x[r].im * F.im;
              Z[i][r].im += x[r].re * F.im + x[r].im * F.re;
              continue;
            }
            // w_c rho_a (P) or w_c rho_b (Q): one word of the element's float2
            const float rho = __builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(
                           fsrc, u * (int)sizeof(float2),
                           ((c * N + bq + 8 * r) * N) * (int)sizeof(float2) + part * (int)sizeof(float), 0));
            if (odd) {   // times i rho
              Z[i][r].re -= x[r].im * rho;
              Z[i][r].im += x[r].re * rho;
            } else {
              Z[i][r].re += x[r].re * rho;
              Z[i][r].im += x[r].im * rho;
            }
          }
        }
      }
      }
      __syncthreads();   // the image is rewritten next
    }
#pragma unroll
    for (int s = 0; s < NQ0; ++s)
#pragma unroll
      for (int r = 0; r < RMAX; ++r) z[s][r] = cmul(z[s][r], (s == 0 && r == 0) ? ratio_e1_lds<NT>[t] : e1[s][r]);
  }

  // ---- inverse transform of the accumulated spectrum: num + i den on the whole window
  if constexpr (MF) {
#pragma unroll
    for (int r = 0; r < M; ++r) tw[r] = mk(tt.re[bq][r], tt.im[bq][r]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) A[(16 * ((wv >> 3) + 2 * i) + mlr) * P + mbq + 8 * (4 * mlq + j)] = Z[i][j];
  } else {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int r = 0; r < M; ++r)
        if (N % LS == 0 || l + LS * i < N) A[(l + LS * i) * P + bq + 8 * r] = Z[i][r];
  }
  __syncthreads();
  pass0_inplace<N, +1, false, N, NT>(A, t, N, true);
  __syncthreads();
  pass1_inplace<N, +1, false, NI, NT>(A, tw, bq, l, N, N);
  __syncthreads();
  pass0_inplace<N, +1, true, N, NT>(A, t, N, true);
  __syncthreads();
  pass1_inplace<N, +1, true, NI, NT>(A, tw, bq, l, N, N);
  __syncthreads();
  // ---- the window index w of a result is the region index (w + R) mod N: region row i'
  // is image row y0 - R + i'; stored along rows, image pixels only
  cx<float>* out = a.part + (long long)blk * N * N;
  const int R = a.R;
  constexpr int NPT = (N * N + NT - 1) / NT;
#pragma unroll 4
  for (int k = 0; k < NPT; ++k) {
    const int e = t + NT * k;
    const int ir = e / N, jr = e - ir * N;
    const int gy = y0 - R + ir, gx = x0 - R + jr;
    if (e < N * N && gy >= 0 && gy < a.ny && gx >= 0 && gx < a.nx) {
      int wy = ir - R, wx = jr - R;
      wy += wy < 0 ? N : 0;
      wx += wx < 0 ? N : 0;
      out[e] = A[wy * P + wx];
    }
  }
}

// 1024 threads: four waves per SIMD at 128 registers (with 512, 212 registers and two
// waves per SIMD measured 1.09 against 0.83 ms for the 2048^2 smoothing). The registers
// hold the accumulator (32), the phases of the thread's four sources (16) and one pass's
// values; the sources' signal values and one phase step per thread sit in the LDS left
// beside the image (16 + 8 KB), which took the spills inside the component loop from 25
// registers to none (0.83 -> 0.69 ms).
template <int N>
constexpr int tratio_threads() {
  return 1024;
}

template <int N, int TV, int PREC, bool PLAIN = false>
__global__ void __launch_bounds__(tratio_threads<N>()) k_tile_ratio(TileRatioArgs a) {
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  const int ntile = a.tx * a.ty;
  ratio_block<N, TV, tratio_threads<N>(), PREC, PLAIN>(a, lb / ntile, lb % ntile, lb, ratio_img_lds<N>);
}

// the plain convolution's gather: out(p) = scale * the sum of the real parts over the
// regions that cover p, in the same fixed order
__global__ void __launch_bounds__(256) k_conv_sum(TileRatioArgs a, int N, float scale) {
  const int px = blockIdx.x * 256 + threadIdx.x, py = blockIdx.y, img = blockIdx.z;
  if (px >= a.nx) return;
  const int T = a.T, R = a.R;
  const int ny0 = py + R - N + 1, nx0 = px + R - N + 1;
  const int by0 = ny0 <= 0 ? 0 : (ny0 + T - 1) / T, by1 = min(a.ty - 1, (py + R) / T);
  const int bx0 = nx0 <= 0 ? 0 : (nx0 + T - 1) / T, bx1 = min(a.tx - 1, (px + R) / T);
  float acc = 0.f;
  for (int by = by0; by <= by1; ++by)
    for (int bx = bx0; bx <= bx1; ++bx) {
      const long long blk = ((long long)img * a.ty + by) * a.tx + bx;
      acc += a.part[(blk * N + (py - by * T + R)) * N + (px - bx * T + R)].re;
    }
  a.y[(long long)img * a.planeY + (long long)py * a.ldY + px] = acc * scale;
}

// out(p) = sum of the real parts over the regions that cover p / the same sum of the
// imaginary parts; the regions are taken in increasing block row, then block column
__global__ void __launch_bounds__(256) k_ratio_sum(TileRatioArgs a, int N) {
  const int px = blockIdx.x * 256 + threadIdx.x, py = blockIdx.y, img = blockIdx.z;
  if (px >= a.nx) return;
  const int T = a.T, R = a.R;
  const int ny0 = py + R - N + 1, nx0 = px + R - N + 1;
  const int by0 = ny0 <= 0 ? 0 : (ny0 + T - 1) / T, by1 = min(a.ty - 1, (py + R) / T);
  const int bx0 = nx0 <= 0 ? 0 : (nx0 + T - 1) / T, bx1 = min(a.tx - 1, (px + R) / T);
  float num = 0.f, den = 0.f;
  for (int by = by0; by <= by1; ++by)
    for (int bx = bx0; bx <= bx1; ++bx) {
      const long long blk = ((long long)img * a.ty + by) * a.tx + bx;
      const cx<float> v = a.part[(blk * N + (py - by * T + R)) * N + (px - bx * T + R)];
      num += v.re;
      den += v.im;
    }
  a.y[(long long)img * a.planeY + (long long)py * a.ldY + px] = num / den;
}

__global__ void __launch_bounds__(256) k_ratio_spectra(const cx<double>* __restrict__ spec, int U, int N,
                                                      const float* __restrict__ w, const float* __restrict__ par,
                                                      float2* __restrict__ out) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long nn = (long long)N * N;
  if (idx >= (long long)U * nn) return;
  const int c = (int)(idx / nn);
  const int rem = (int)(idx - (long long)c * nn);
  const int v = rem / N, u = rem - v * N;   // output [c][v][u]
  const cx<double>* S = spec + (long long)c * nn;
  const cx<double> F = S[(long long)u * N + v];
  const cx<double> Fm = S[(long long)((N - u) % N) * N + (N - v) % N];
  // spectrum of Re F_c: (F(w) + conj F(-w)) / 2; of Im F_c: (F(w) - conj F(-w)) / (2i)
  const double ar = 0.5 * (F.re + Fm.re), ai = 0.5 * (F.im - Fm.im);
  const double dr = 0.5 * (F.re - Fm.re), di = 0.5 * (F.im + Fm.im);
  const double br = di, bi = -dr;
  const bool odd = par[c] < 0.f;
  const double wc = (double)w[c];
  out[idx] = make_float2((float)(wc * (odd ? ai : ar)), (float)(wc * (odd ? bi : br)));
}

}  // namespace

hipError_t launch_ratio_spectra(hipStream_t s, const cx<double>* spec, int U, int N, const float* w,
                                const float* par, float2* out) {
  const long long n = (long long)U * N * N;
  hipLaunchKernelGGL(k_ratio_spectra, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, spec, U, N, w, par, out);
  return last();
}

// N = 128 only: for radii up to 16 (N = 96 blocks) the two launches of the overlap-save
// block convolution measured faster (1024^2, 31 x 31, K = 16: 0.153 against 0.204 ms)
#define ECC_TRATIO_CONFIGS(X) X(128, 64)

bool tratio_supported(int N, int TV) {
#define ECC_RS(n, tv) if (N == n && TV == tv) return true;
  ECC_TRATIO_CONFIGS(ECC_RS)
#undef ECC_RS
  return false;
}

size_t tratio_scratch_bytes(int N, int T, int batch, int ny, int nx) {
  const long long nblk = (long long)((ny + T - 1) / T) * ((nx + T - 1) / T) * batch;
  return (size_t)nblk * N * N * sizeof(cx<float>);
}

hipError_t launch_tile_ratio(hipStream_t s, int N, int TV, int batch, const TileRatioArgs& a0, int prec, bool plain) {
  TileRatioArgs a = a0;
  if (a.T < 1 || a.T > TV || a.T + 2 * a.R > N || a.R < 0 || prec < 0 || prec > 2) return hipErrorInvalidValue;
  if (plain && prec != 0) return hipErrorInvalidValue;
  a.tx = (a.nx + a.T - 1) / a.T;
  a.ty = (a.ny + a.T - 1) / a.T;
  const long long nblk = (long long)a.tx * a.ty * batch;
  if (nblk > 0x7fffffffLL || a.ny > 65535 || batch > 65535) return hipErrorInvalidValue;
#define ECC_RL(n, tv)                                                                                 \
  if (N == n && TV == tv) {                                                                          \
    if (plain) {                                                                                     \
      hipLaunchKernelGGL((k_tile_ratio<n, tv, 0, true>), dim3((unsigned)nblk), dim3(tratio_threads<n>()), 0, s, \
                         a);                                                                         \
      hipError_t e = last();                                                                         \
      if (e != hipSuccess) return e;                                                                 \
      hipLaunchKernelGGL(k_conv_sum, dim3((unsigned)((a.nx + 255) / 256), (unsigned)a.ny, (unsigned)batch), \
                         dim3(256), 0, s, a, n, 1.0f / ((float)n * (float)n));                       \
      return last();                                                                                 \
    }                                                                                                \
    if (prec == 0)                                                                                   \
      hipLaunchKernelGGL((k_tile_ratio<n, tv, 0>), dim3((unsigned)nblk), dim3(tratio_threads<n>()), 0, s, a); \
    else if (prec == 1)                                                                              \
      hipLaunchKernelGGL((k_tile_ratio<n, tv, 1>), dim3((unsigned)nblk), dim3(tratio_threads<n>()), 0, s, a); \
    else                                                                                             \
      hipLaunchKernelGGL((k_tile_ratio<n, tv, 2>), dim3((unsigned)nblk), dim3(tratio_threads<n>()), 0, s, a); \
    hipError_t e = last();                                                                           \
    if (e != hipSuccess) return e;                                                                   \
    hipLaunchKernelGGL(k_ratio_sum, dim3((unsigned)((a.nx + 255) / 256), (unsigned)a.ny, (unsigned)batch), \
                       dim3(256), 0, s, a, n);                                                       \
    return last();                                                                                   \
  }
  ECC_TRATIO_CONFIGS(ECC_RL)
#undef ECC_RL
  return hipErrorInvalidValue;
}

}  // namespace ecc
