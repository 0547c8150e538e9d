// Tiled (overlap-save) extended correlation: every workgroup owns one T x T block of
// output pixels and keeps the whole computation for it on chip.
//
// The block's N x N input window (rows y0 - R .. y0 - R + N - 1, same for columns; zero
// outside the image) is transformed once. For each component c the product
// hhat * conj(fhat_c) is transformed back, and since the filter spectrum fhat_c belongs to
// F_c placed at window offset (R, R) -> (0, 0) .. (2R, 2R), circular index (u, x) of the
// result equals the linear correlation (H star F_c)(y0 + u, x0 + x) for u, x < N - 2R:
// the cyclic wrap only touches indices past the valid block. The components are then
// combined per pixel with e^{i (kofs + c) alpha(p)} exactly as in the two-pass form
// (section 4, extended correlation by Fourier-domain products), so the only global
// traffic is the signal window, the angle field, the output and the (L2-resident)
// filter spectra.
//
// Transforms have length N = 8 * M (M = 8, 12, 16), done as two Stockham passes:
// pass 0 radix 8 (M butterflies per line, in[b + M r] -> out[8 b + r]), pass 1 radix M
// (8 butterflies per line, in[b + 8 r] -> out[b + 8 r] after the twiddle w^{r b}, so the
// last pass works in place). A 2D transform is a column pass pair then a row pass pair
// on an LDS image of N rows with an odd pitch (conflict-free both along rows and
// columns). Only the T valid rows are carried from the column to the row transforms.
#include "tile_common.hpp"

namespace ecc {

namespace {

// One block (image img, block index `tile`) with one group of NT threads (256 or 512),
// components one after another. N: transform length; TV: largest valid block side (a
// multiple of 32); SEPB: the row pass-0 output goes to a second buffer of TV rows (else
// in place, one more barrier); STACK: write the components instead of combining them.
// LS = NT / 8 threads share each pass-1 butterfly index (with 512 threads it is the wave
// index, so the twiddles are scalar). Called by every thread of the workgroup.
//
// SYM (rotation filters, N = 128, 512 threads): centred spectra and mirror items as in the
// pair form below; thread t does mirror pairs t and 512 + t (t < 510), threads 510 and 511
// do two of the four self-mirrored items through the same code (the mirror of such an item
// is the item itself, so the second transform rewrites the same values), and the other two
// are single units of lanes in waves 0 and 1.
template <int N, int TV, bool SEPB, bool STACK = false, int NT = kTileThreads, bool SYM = false>
__device__ __forceinline__ void corr_block_one(const TileArgs& a, int img, int tile, cx<float>* lds_t,
                                               int tid = -1) {
  static_assert(!SYM || (N == 128 && NT == 512 && !SEPB), "symmetric one-group form: N = 128, 512 threads");
  constexpr int M = N / 8, P = N + 1, LS = NT / 8;
  constexpr int NQ0 = (N * M + NT - 1) / NT;   // column pass-0 items
  constexpr int NQ2 = (TV * M + NT - 1) / NT;  // row pass-0 items
  constexpr int TR = (TV + LS - 1) / LS, RV = TV / 8;
  constexpr bool PREFETCH = NT == kTileThreads && N <= 96;
  const int t = tid >= 0 ? tid : (int)threadIdx.x, l = t % LS;
  const int bq = NT == 512 ? __builtin_amdgcn_readfirstlane(t / LS) : t / LS;
  cx<float>* A = lds_t;
  cx<float>* Bb = SEPB ? A + N * P : A;
  const int y0 = (tile / a.tx) * a.T, x0 = (tile % a.tx) * a.T;
  const int T = a.T;

  cx<float> tw[M];
  {
    const TileTwiddles<N>& tt = tile_twiddles<N>();
#pragma unroll
    for (int r = 0; r < M; ++r) tw[r] = mk(tt.re[bq][r], tt.im[bq][r]);
  }

  __syncthreads();   // the LDS image may still be in use by the previous block
  // field values of the block, loaded just before the window (so that the two latencies
  // overlap) with consecutive lanes along rows; they reach the threads that own the pixels
  // (rows l + LS i, columns bq + 8 r) through LDS below
  constexpr int FPT = (TV * TV + NT - 1) / NT, FL = TV + 1;   // per thread; LDS pitch
  float fco[STACK ? 1 : FPT];
  if constexpr (!STACK) {
#pragma unroll
    for (int k = 0; k < FPT; ++k) {
      const int e = t + NT * k, row = e / TV, col = e % TV;
      const int gy = y0 + row, gx = x0 + col;
      fco[k] = (e < TV * TV && row < T && col < T && gy < a.ny && gx < a.nx)
                   ? a.fld.ptr[(long long)img * a.fld.plane + (long long)gy * a.fld.ld + gx]
                   : 0.f;
    }
  }
  // ---- forward 2D transform of the signal window
  forward_window<N, NT>(A, a.H + (long long)img * a.planeH, a.ldH, a.ny, a.nx, y0, x0, a.R, t);
  // signal spectrum values of this thread's column pass-0 items, kept for all components
  constexpr int NHS = SYM ? 3 : NQ0;
  cx<float> hs[NHS][8];
  int sv[SYM ? 3 : 1], sb[SYM ? 3 : 1];   // SYM: items of slots A, B, C
  if constexpr (SYM) {
    // canonical item of pair p: b in 1 .. M/2 - 1 (all columns), then b = M/2 and b = 0
    // with columns 1 .. N/2 - 1
    constexpr int NB = (M / 2 - 1) * N, NPAIR = (N * M - 4) / 2;
    static_assert(NPAIR == 2 * NT - 2, "pair count");
    auto pair_item = [&](int p, int& v, int& b) {
      if (p < NB) {
        b = 1 + p / N;
        v = p % N;
      } else {
        const int p2 = p - NB;
        b = p2 < N / 2 - 1 ? M / 2 : 0;
        v = 1 + (p2 < N / 2 - 1 ? p2 : p2 - (N / 2 - 1));
      }
    };
    auto self_item = [&](int f, int& v, int& b) {
      v = (f & 1) * (N / 2);
      b = (f >> 1) * (M / 2);
    };
    pair_item(t, sv[0], sb[0]);
    if (t < NT - 2) pair_item(NT + t, sv[1], sb[1]);
    else self_item(t - (NT - 2), sv[1], sb[1]);
    self_item(t == 127 ? 3 : 2, sv[2], sb[2]);
    const TilePhases<N>& ph = tile_phases<N>();
    const int ms = (M * a.R) % N;
    const cx<float> step = mk(ph.re[ms], ph.im[ms]);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int m0 = ((sb[s] + sv[s]) * a.R) % N;
      cx<float> pr = mk(ph.re[m0], ph.im[m0]);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        hs[s][r] = cmul(window_spectrum<N>(A, sb[s] + M * r, sv[s]), pr);
        pr = cmul(pr, step);
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < NQ0; ++s) {
      const int q = t + s * NT;
      const int v = q % N, b = q / N;
#pragma unroll
      for (int r = 0; r < 8; ++r) hs[s][r] = (b < M) ? window_spectrum<N>(A, b + M * r, v) : mk(0.f, 0.f);
    }
  }
  float fvs[STACK ? 1 : TR][RV];
  if constexpr (!STACK) {
    float* fl = reinterpret_cast<float*>(A);
    __syncthreads();   // the spectrum reads above are done
#pragma unroll
    for (int k = 0; k < FPT; ++k) {
      const int e = t + NT * k;
      if (e < TV * TV) fl[(e / TV) * FL + e % TV] = fco[k];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
      for (int r = 0; r < RV; ++r) {
        const int u = l + LS * i;
        fvs[i][r] = u < TV ? fl[u * FL + bq + 8 * r] : 0.f;
      }
  }

  // ---- per-pixel state of the row pass-1 outputs: pixel (l + LS i, bq + 8 r). The
  // phase of component c is e^{i (kofs + c) alpha}, advanced by one factor e^{i alpha}
  // per component.
  float acc[TR][RV];
  cx<float> z[TR][RV], e1[TR][RV];
#pragma unroll
  for (int i = 0; i < TR; ++i) {
#pragma unroll
    for (int r = 0; r < RV; ++r) {
      acc[i][r] = 0.f;
      z[i][r] = mk(0.f, 0.f);
      e1[i][r] = mk(0.f, 0.f);
      const int u = l + LS * i, x = bq + 8 * r;
      const int gy = y0 + u, gx = x0 + x;
      if (!STACK && u < T && x < T && gy < a.ny && gx < a.nx) {
        const float fv = fvs[STACK ? 0 : i][r];
        const int k0 = a.kofs;
        cx<float> s1, s0;
        if (a.fld.log_mode || a.kofs != 0) {
          const double al = field_angle(a.fld, fv);
          double sn, cs;
          sincos(al, &sn, &cs);
          s1 = mk((float)cs, (float)sn);
          sincos((double)k0 * al, &sn, &cs);
          s0 = mk((float)cs, (float)sn);
        } else {
          const float al = (float)a.fld.mul * fv + (float)a.fld.add;
          float sn, cs;
          sincosf(al, &sn, &cs);
          s1 = mk(cs, sn);
          s0 = mk(1.f, 0.f);
        }
        z[i][r] = s0;
        e1[i][r] = s1;
      }
    }
  }

  // filter spectrum values of the first component (prefetching form)
  cx<float> fs[PREFETCH ? NQ0 : 1][8];
  if constexpr (PREFETCH) {
#pragma unroll
    for (int s = 0; s < NQ0; ++s) {
      const int q = t + s * NT;
      const int v = q % N, b = q / N;
#pragma unroll
      for (int r = 0; r < 8; ++r) fs[s][r] = (b < M) ? a.Fs[(b + M * r) * N + v] : mk(0.f, 0.f);
    }
  }
  __syncthreads();   // A is rewritten below

  for (int c = 0; c < a.U; ++c) {
    const bool act = c < a.U;
    // ---- column pass 0: product, inverse radix 8, A[8 b + r][v]
    const cx<float>* Fc = a.Fs + (long long)c * N * N;
    const bool more = c + 1 < a.U;
    // without the register prefetch, the pass's filter-spectrum loads are issued in two
    // groups of items ahead of their products (a latency per group, not per item)
    constexpr int GQ = PREFETCH ? 1 : (NQ0 + 1) / 2;
    if constexpr (SYM) {
      const float par = (c & 1) ? -1.f : 1.f;   // (-1)^c (components from offset 0)
      auto unit = [&](int s, bool pair, bool maybe_b0) {
        const int v = sv[s], b = sb[s];
        cx<float> f[8], x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) f[r] = Fc[(b + M * r) * N + v];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = cmulc(hs[s][r], f[r]);
        dft<8, +1, float>(x);
#pragma unroll
        for (int r = 0; r < 8; ++r) A[(8 * b + r) * P + v] = x[r];
        if (pair) {
          cx<float> g[8], y[8];
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const cx<float> hf = cmul(hs[s][r], f[r]);
            g[r] = mk(par * hf.re, -par * hf.im);
          }
#pragma unroll
          for (int j = 0; j < 8; ++j) y[j] = (maybe_b0 && b == 0) ? g[(8 - j) & 7] : g[7 - j];
          dft<8, +1, float>(y);
          const int vm = v == 0 ? 0 : N - v, bm = b == 0 ? 0 : M - b;
#pragma unroll
          for (int r = 0; r < 8; ++r) A[(8 * bm + r) * P + vm] = y[r];
        }
      };
      unit(0, true, false);
      unit(1, true, true);
      if (t == 63 || t == 127) unit(2, false, false);
    } else
#pragma unroll
    for (int s0 = 0; s0 < NQ0; s0 += GQ) {
      cx<float> fl[GQ][8];
      if constexpr (!PREFETCH) {
#pragma unroll
        for (int g2 = 0; g2 < GQ; ++g2) {
          const int q = t + (s0 + g2) * NT;
          const int v = q % N, b = q / N;
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            fl[g2][r] = mk(0.f, 0.f);
            if (s0 + g2 < NQ0 && act && b < M) fl[g2][r] = Fc[(b + M * r) * N + v];
          }
        }
      }
#pragma unroll
      for (int g2 = 0; g2 < GQ; ++g2) {
        const int s = s0 + g2;
        const int q = t + s * NT;
        const int v = q % N, b = q / N;
        if (s < NQ0 && act && b < M) {
          cx<float> x[8];
          if constexpr (PREFETCH) {
#pragma unroll
            for (int r = 0; r < 8; ++r) x[r] = cmulc(hs[s][r], fs[s][r]);
            if (more) {
#pragma unroll
              for (int r = 0; r < 8; ++r) fs[s][r] = Fc[N * N + (b + M * r) * N + v];   // next component
            }
          } else {
#pragma unroll
            for (int r = 0; r < 8; ++r) x[r] = cmulc(hs[s][r], fl[g2][r]);
          }
          dft<8, +1, float>(x);
#pragma unroll
          for (int r = 0; r < 8; ++r) A[(8 * b + r) * P + v] = x[r];
        }
      }
    }
    __syncthreads();
    // ---- column pass 1 (in place), rows < T kept
    if (act) pass1_inplace<N, +1, false, N / LS, NT, TV / 8>(A, tw, bq, l, N, T);
    __syncthreads();
    // ---- row pass 0 over the T valid rows
    if constexpr (SEPB) {
#pragma unroll
      for (int s = 0; s < NQ2; ++s) {
        const int q = t + s * NT;
        const int u = q % TV, b = q / TV;
        if (act && b < M && u < T) {
          cx<float> x[8];
#pragma unroll
          for (int r = 0; r < 8; ++r) x[r] = A[u * P + b + M * r];
          dft<8, +1, float>(x);
#pragma unroll
          for (int r = 0; r < 8; ++r) Bb[u * P + 8 * b + r] = x[r];
        }
      }
    } else {
      pass0_inplace<N, +1, true, TV, NT>(A, t, T, act);
    }
    __syncthreads();
    // ---- row pass 1 and the per-pixel combination
    if (act) {
      const float wc = a.w[c];
#pragma unroll
      for (int i = 0; i < TR; ++i) {   // (acc, z, e1 are indexed by i: this loop stays unrolled)
        const int u = l + LS * i;
        if (u < T) {
          cx<float> x[M];
#pragma unroll
          for (int r = 0; r < M; ++r) x[r] = Bb[u * P + bq + 8 * r];
#pragma unroll
          for (int r = 1; r < M; ++r) x[r] = cmul(x[r], tw[r]);
          dft<M, +1, float>(x);
          if constexpr (STACK) {
            // back into the image (the positions this thread read), stored below along rows
#pragma unroll
            for (int r = 0; r < RV; ++r) Bb[u * P + bq + 8 * r] = x[r];
          } else {
#pragma unroll
            for (int r = 0; r < RV; ++r) {
              acc[i][r] += wc * (z[i][r].re * x[r].re - z[i][r].im * x[r].im);
              z[i][r] = cmul(z[i][r], e1[i][r]);
            }
          }
        }
      }
    }
    // A is rewritten by the next column pass (stack form: a barrier for LDS only, so that
    // this component's stack stores are not waited for)
    if constexpr (STACK) {
      // the T x T block of G_c, with consecutive lanes along rows
      __syncthreads();
      float* dst = a.stack + 2 * (long long)c * a.stack_plane;
#pragma unroll
      for (int k = 0; k < FPT; ++k) {
        const int e = t + NT * k, row = e / TV, col = e % TV;
        const int gy = y0 + row, gx = x0 + col;
        if (e < TV * TV && row < T && col < T && gy < a.ny && gx < a.nx) {
          const cx<float> v = Bb[row * P + col];
          *reinterpret_cast<float2*>(dst + 2 * ((long long)(gy - a.stack_y0) * a.nx + gx)) =
              make_float2(v.re * a.scale, v.im * a.scale);
        }
      }
      lds_barrier();   // the image is rewritten next; the stores are not waited for
    } else if constexpr (!SEPB) {
      __syncthreads();   // A is rewritten by the next column pass
    }
  }

  if constexpr (!STACK) {
    // outputs through LDS, then stored along rows
    float* ob = reinterpret_cast<float*>(A);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TR; ++i) {
#pragma unroll
      for (int r = 0; r < RV; ++r) {
        const int u = l + LS * i;
        if (u < TV) ob[u * FL + bq + 8 * r] = acc[i][r] * a.scale;
      }
    }
    __syncthreads();
    float* yb = a.y + (long long)img * a.planeY;
    // (the thread index through a lane shuffle: the compiler would otherwise keep the
    // field loads' addresses, which are the same expressions, live through the loop)
    const int ts = __shfl(t, t & 63);
#pragma unroll
    for (int k = 0; k < FPT; ++k) {
      const int e = ts + NT * k, row = e / TV, col = e % TV;
      const int gy = y0 + row, gx = x0 + col;
      if (e < TV * TV && row < T && col < T && gy < a.ny && gx < a.nx) yb[(long long)gy * a.ldY + gx] = ob[row * FL + col];
    }
  }
}

// Component pairs: 512 threads transform components c and c + 1 side by side, each in
// its own LDS image (A[0], A[1]); TV = 64.
//  * column pass 0: item (v, b) (column v, radix-8 butterfly b) is done for both
//    components by the same thread, so a thread keeps the signal spectrum of its items
//    once; items q < 512 NF are full (both components), the remaining REM items are
//    dealt as single-component halves to threads t < 2 REM (per SIMD the load is equal).
//  * column passes 1 and row passes 0: group g = t / 256 works on component c + g.
//  * row pass 1: thread (row u = t mod 64, butterfly bq = t / 64) does both components;
//    bq is uniform in a wave, so its twiddles come from scalar loads, and the thread owns
//    the 8 pixels (u, bq + 8 r) for all components.
//
// SYM (rotation filters, N = 96): the spectra are those of the centred components F~_c
// (offset x at x mod N), for which F~_c(-w) = (-1)^c F~_c(w); the window spectrum is taken
// as h'(w) = h(w) e^{2 pi i (w_y + w_x) R / N}, which gives the same products
// h'(w) conj(F~_c(w)) = h(w) conj(f_c(w)) and satisfies h'(-w) = conj(h'(w)) (real
// window). A thread then does an item and its mirror item (column -v, rows -k) from one
// set of filter-spectrum loads: the mirror products are (-1)^c conj(h'(w) F~_c(w)), which
// halves the spectrum reads of column pass 0.
//
// Y2: also accumulate sum_c w_c (kofs + c) Im(z_c G_c) and write it times mulsig as the
// second output y2 (the field part of the adjoint).
template <int N, bool STACK = false, bool SYM = false, bool Y2 = false>
__device__ __forceinline__ void corr_block_pair(const TileArgs& a, int img, int tile, cx<float>* lds_t,
                                                int tid = -1) {
  constexpr int M = N / 8, P = N + 1, TV = 64, NL = N * M;
  constexpr int NF = NL / (2 * kTileThreads), REM = NL - NF * 2 * kTileThreads;
  constexpr int NH = SYM ? 2 : NF + (REM ? 1 : 0);
  // SYM: item pairs (item, mirror) apart from the 4 self-mirrored items (v in {0, N/2},
  // b in {0, M/2}); thread t does pair t for both components, and the remaining pairs and
  // the self-mirrored items are dealt as single-component units to threads t < NX
  constexpr int NPAIR = (NL - 4) / 2, NX = 2 * (NPAIR - 2 * kTileThreads) + 8;
  static_assert(!SYM || (N == 96 && NPAIR >= 2 * kTileThreads && NX <= 2 * kTileThreads),
                "symmetric pair form: N = 96");
  static_assert(REM * 2 <= 2 * kTileThreads, "remainder items exceed one round");
  const int t = tid >= 0 ? tid : (int)threadIdx.x;
  const int g = t / kTileThreads, tg = t - g * kTileThreads;
  const int bq1 = tg >> 5, l1 = tg & 31;                       // column pass 1 mapping
  const int u4 = t & 63;
  const int bq4 = __builtin_amdgcn_readfirstlane(t >> 6);      // row pass 1 mapping
  cx<float>* const A0 = lds_t;
  cx<float>* const A1 = lds_t + N * P;
  cx<float>* const Ag = g ? A1 : A0;
  const int y0 = (tile / a.tx) * a.T, x0 = (tile % a.tx) * a.T;
  const int T = a.T;
  const TileTwiddles<N>& tt = tile_twiddles<N>();

  cx<float> tw1[M];
#pragma unroll
  for (int r = 0; r < M; ++r) tw1[r] = mk(tt.re[bq1][r], tt.im[bq1][r]);

  __syncthreads();   // the LDS images may still be in use by the previous block
  // field values of the block, loaded just before the window (so that the two latencies
  // overlap) with consecutive lanes along rows; they reach the threads that own the pixels
  // (row u4, columns bq4 + 8 r) through LDS below
  const bool rowok = u4 < T && y0 + u4 < a.ny;
  constexpr int FPT = TV * TV / (2 * kTileThreads), FL = TV + 1;   // per thread; LDS pitch
  float fco[STACK ? 1 : FPT];
  if constexpr (!STACK) {
#pragma unroll
    for (int i = 0; i < FPT; ++i) {
      const int e = t + 2 * kTileThreads * i, row = e / TV, col = e % TV;
      const int gy = y0 + row, gx = x0 + col;
      fco[i] = (row < T && col < T && gy < a.ny && gx < a.nx)
                   ? a.fld.ptr[(long long)img * a.fld.plane + (long long)gy * a.fld.ld + gx]
                   : 0.f;
    }
  }
  // ---- forward transform of the signal window, by all 512 threads on image A0 (A1 is
  // only the working image of the second component). While the window loads are in
  // flight the field values go to A1 (free until the component loop), in the common case
  // (angle field, components from k = 0) already as the phase step e^{i alpha}; the
  // transform's barriers order these writes before the reads below.
  const bool fast = !a.fld.log_mode && a.kofs == 0;
  auto stage_field = [&]() {
    if constexpr (!STACK) {
      float2* fl = reinterpret_cast<float2*>(A1);
#pragma unroll
      for (int i = 0; i < FPT; ++i) {
        const int e = t + 2 * kTileThreads * i;
        float2 v = make_float2(fco[i], 0.f);
        if (fast) {
          float sn, cs;
          sincosf((float)a.fld.mul * fco[i] + (float)a.fld.add, &sn, &cs);
          v = make_float2(cs, sn);
        }
        fl[(e / TV) * FL + e % TV] = v;
      }
    }
  };
  forward_window<N, 2 * kTileThreads>(A0, a.H + (long long)img * a.planeH, a.ldH, a.ny, a.nx, y0, x0, a.R, t,
                                      0, 0, stage_field);
  float2 fvs[8];
  if constexpr (!STACK) {
    const float2* fl = reinterpret_cast<const float2*>(A1);
#pragma unroll
    for (int r = 0; r < 8; ++r) fvs[r] = fl[u4 * FL + bq4 + 8 * r];
  }
  // signal spectrum of this thread's column pass-0 items
  cx<float> hs[NH][8];
  int qv[NH], qb[NH];
  int hcomp = 0;      // component of the half item (t < 2 REM), or of the extra unit (SYM)
  bool xpair = false;  // SYM: the extra unit is an item pair (else a self-mirrored item)
  if constexpr (SYM) {
    // canonical item of pair p: b in 1 .. M/2 - 1 (all columns), then b = M/2 and b = 0
    // with columns 1 .. N/2 - 1 (the b = 0 pairs, whose mirror order differs, come last
    // and so fall to the extra units only)
    auto pair_item = [&](int p, int& v, int& b) {
      constexpr int NB = (M / 2 - 1) * N;
      if (p < NB) {
        b = 1 + p / N;
        v = p % N;
      } else {
        const int p2 = p - NB;
        b = p2 < N / 2 - 1 ? M / 2 : 0;
        v = 1 + (p2 < N / 2 - 1 ? p2 : p2 - (N / 2 - 1));
      }
    };
    static_assert((M / 2 - 1) * N + N / 2 - 1 >= 2 * kTileThreads, "b = 0 pairs beyond the base units");
    pair_item(t, qv[0], qb[0]);
    const int e = t < NX ? t : 0;
    hcomp = e & 1;
    xpair = e < 2 * (NPAIR - 2 * kTileThreads);
    if (xpair) {
      pair_item(2 * kTileThreads + e / 2, qv[1], qb[1]);
    } else {
      const int sf = (e - 2 * (NPAIR - 2 * kTileThreads)) / 2;
      qv[1] = (sf & 1) * (N / 2);
      qb[1] = (sf >> 1) * (M / 2);
    }
    // the phase e^{2 pi i (k + v) R / N} of element r (row k = b + M r) advances by the
    // uniform factor e^{2 pi i M R / N} from r to r + 1: one table read per item
    const TilePhases<96>& ph = kPh96;
    const int ms = (M * a.R) % N;
    const cx<float> step = mk(ph.re[ms], ph.im[ms]);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int m0 = ((qb[s] + qv[s]) * a.R) % N;
      cx<float> pr = mk(ph.re[m0], ph.im[m0]);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        hs[s][r] = cmul(window_spectrum<N>(A0, qb[s] + M * r, qv[s]), pr);
        pr = cmul(pr, step);
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < NH; ++s) {
      int q = t + s * 2 * kTileThreads;
      if (s == NF) q = NF * 2 * kTileThreads + (REM ? t % (REM ? REM : 1) : 0);
      qv[s] = q % N;
      qb[s] = q / N;
      const bool ok = s < NF || t < 2 * REM;
#pragma unroll
      for (int r = 0; r < 8; ++r) hs[s][r] = ok ? window_spectrum<N>(A0, qb[s] + M * r, qv[s]) : mk(0.f, 0.f);
    }
    hcomp = REM ? t / (REM ? REM : 1) : 0;
  }

  // ---- per-pixel state: pixel (u4, bq4 + 8 r), phase e^{i (kofs + c) alpha}
  float acc[8], acc2[Y2 ? 8 : 1];
  cx<float> z[8], e1[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    acc[r] = 0.f;
    if constexpr (Y2) acc2[r] = 0.f;
    z[r] = mk(0.f, 0.f);
    e1[r] = mk(0.f, 0.f);
    const int x = bq4 + 8 * r, gx = x0 + x;
    if (!STACK && rowok && x < T && gx < a.nx) {
      const float fv = fvs[r].x;
      if (fast) {   // staged as e^{i alpha}
        e1[r] = mk(fvs[r].x, fvs[r].y);
        z[r] = mk(1.f, 0.f);
      } else {      // staged as the field value: log-scale angle or components from kofs
        const double al = field_angle(a.fld, fv);
        double sn, cs;
        sincos(al, &sn, &cs);
        e1[r] = mk((float)cs, (float)sn);
        sincos((double)a.kofs * al, &sn, &cs);
        z[r] = mk((float)cs, (float)sn);
      }
    }
  }
  __syncthreads();   // the images are rewritten below

  for (int c = 0; c < a.U; c += 2) {
    const bool two = c + 1 < a.U;
    const cx<float>* F0 = a.Fs + (long long)c * N * N;
    // ---- column pass 0 for both components
    if constexpr (SYM) {
      // unit: slot s (0: this thread's pair, both components; 1: the extra unit), component cc
      auto unit = [&](int s, int cc, bool pair, float par, bool maybe_b0) {
        const int v = qv[s], b = qb[s];
        const cx<float>* Fc = F0 + cc * N * N;
        cx<float>* Ac = cc ? A1 : A0;
        cx<float> f[8], x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) f[r] = Fc[(b + M * r) * N + v];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = cmulc(hs[s][r], f[r]);
        dft<8, +1, float>(x);
#pragma unroll
        for (int r = 0; r < 8; ++r) Ac[(8 * b + r) * P + v] = x[r];
        if (pair) {
          // mirror item (column -v, butterfly -b mod M): its element r' holds row -(b + M r),
          // r' = 7 - r for b > 0 and (8 - r) mod 8 for b = 0
          cx<float> g[8], y[8];
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const cx<float> hf = cmul(hs[s][r], f[r]);
            g[r] = mk(par * hf.re, -par * hf.im);
          }
#pragma unroll
          for (int j = 0; j < 8; ++j) y[j] = (maybe_b0 && b == 0) ? g[(8 - j) & 7] : g[7 - j];
          dft<8, +1, float>(y);
          const int vm = v == 0 ? 0 : N - v, bm = b == 0 ? 0 : M - b;
#pragma unroll
          for (int r = 0; r < 8; ++r) Ac[(8 * bm + r) * P + vm] = y[r];
        }
      };
      unit(0, 0, true, 1.f, false);
      if (two) unit(0, 1, true, -1.f, false);
      if (t < NX && (hcomp == 0 || two)) unit(1, hcomp, xpair, hcomp ? -1.f : 1.f, true);
    } else
#pragma unroll
    for (int s = 0; s < NH; ++s) {
      const bool full = s < NF;
      if (full || t < 2 * REM) {
        const int v = qv[s], b = qb[s];
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
          const bool mine = full ? (cc == 0 || two) : (cc == hcomp && (cc == 0 || two));
          if (mine) {
            const cx<float>* Fc = F0 + cc * N * N;
            cx<float> x[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) x[r] = cmulc(hs[s][r], Fc[(b + M * r) * N + v]);
            dft<8, +1, float>(x);
            cx<float>* Ac = cc ? A1 : A0;
#pragma unroll
            for (int r = 0; r < 8; ++r) Ac[(8 * b + r) * P + v] = x[r];
          }
        }
      }
    }
    __syncthreads();
    // ---- column pass 1 (in place, rows < T kept) and row pass 0, group g on c + g; at
    // N = 96 a last odd component is shared by both groups (columns, then rows, split in
    // halves)
    if (N != 96 || two) {
      if (g == 0 || two) pass1_inplace<N, +1, false, N / 32, kTileThreads, TV / 8>(Ag, tw1, bq1, l1, N, T);
    } else {
      constexpr int HN = N / 2;
      pass1_inplace<N, +1, false, (HN + 31) / 32, kTileThreads, TV / 8>(A0 + g * HN, tw1, bq1, l1, HN, T);
    }
    __syncthreads();
    if (N != 96 || two) {
      pass0_inplace<N, +1, true, TV>(Ag, tg, T, g == 0 || two);
    } else {
      constexpr int HT = TV / 2;
      const int nl = g ? T - HT : (T < HT ? T : HT);
      pass0_inplace<N, +1, true, HT>(A0 + g * HT * P, tg, nl, nl > 0);
    }
    __syncthreads();
    // ---- row pass 1 for both components and the per-pixel combination
    if (u4 < T) {
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        if (cc == 0 || two) {
          const cx<float>* Ac = cc ? A1 : A0;
          cx<float> x[M];
#pragma unroll
          for (int r = 0; r < M; ++r) x[r] = Ac[u4 * P + bq4 + 8 * r];
#pragma unroll
          for (int r = 1; r < M; ++r) x[r] = cmul(x[r], mk(tt.re[bq4][r], tt.im[bq4][r]));
          dft<M, +1, float>(x);
          if constexpr (STACK) {
            // back into the image (the positions this thread read), stored below along rows
            cx<float>* Aw = cc ? A1 : A0;
#pragma unroll
            for (int r = 0; r < 8; ++r) Aw[u4 * P + bq4 + 8 * r] = x[r];
          } else {
            const float wc = a.w[c + cc];
            const float wk = Y2 ? wc * (float)(a.kofs + c + cc) : 0.f;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
              acc[r] += wc * (z[r].re * x[r].re - z[r].im * x[r].im);
              if constexpr (Y2) acc2[r] += wk * (z[r].re * x[r].im + z[r].im * x[r].re);
              z[r] = cmul(z[r], e1[r]);
            }
          }
        }
      }
    }
    if constexpr (STACK) {
      // the pair's T x T blocks of G_c and G_{c+1}, with consecutive lanes along rows
      __syncthreads();
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        if (cc == 0 || two) {
          const cx<float>* Ar = cc ? A1 : A0;
          float* dst = a.stack + 2 * (long long)(c + cc) * a.stack_plane;
#pragma unroll
          for (int i = 0; i < FPT; ++i) {
            const int e = t + 2 * kTileThreads * i, row = e / TV, col = e % TV;
            const int gy = y0 + row, gx = x0 + col;
            if (row < T && col < T && gy < a.ny && gx < a.nx) {
              const cx<float> v = Ar[row * P + col];
              *reinterpret_cast<float2*>(dst + 2 * ((long long)(gy - a.stack_y0) * a.nx + gx)) =
                  make_float2(v.re * a.scale, v.im * a.scale);
            }
          }
        }
      }
      lds_barrier();   // the images are rewritten next; the stores are not waited for
    } else {
      __syncthreads();   // the images are rewritten by the next column pass
    }
  }

  if constexpr (!STACK) {
    // outputs through LDS (free after the last barrier), then stored along rows
    float* ob = reinterpret_cast<float*>(A0);
    float* ob2 = reinterpret_cast<float*>(A1);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      ob[u4 * FL + bq4 + 8 * r] = acc[r] * a.scale;
      if constexpr (Y2) ob2[u4 * FL + bq4 + 8 * r] = acc2[r] * a.scale;
    }
    __syncthreads();
    float* yb = a.y + (long long)img * a.planeY;
    // (the thread index through a lane shuffle: the compiler would otherwise keep the
    // field loads' addresses, which are the same expressions, live through the loop)
    const int ts = __shfl(t, t & 63);
#pragma unroll
    for (int i = 0; i < FPT; ++i) {
      const int e = ts + 2 * kTileThreads * i, row = e / TV, col = e % TV;
      const int gy = y0 + row, gx = x0 + col;
      if (row < T && col < T && gy < a.ny && gx < a.nx) {
        yb[(long long)gy * a.ldY + gx] = ob[row * FL + col];
        if constexpr (Y2)
          a.y2[(long long)img * a.planeY + (long long)gy * a.ldY + gx] =
              ob2[row * FL + col] * a.mulsig[(long long)img * a.planeMul + (long long)gy * a.ldMul + gx];
      }
    }
  }
}

// Threads of a launch: the pair form has 2 x 256; the one-group form 512 for N = 128
// (every pass divides evenly, and two waves per SIMD hide latency) and 256 otherwise.
template <int N, int HV>
constexpr int tile_nt() {
  return HV == 2 ? 2 * kTileThreads : (N == 128 ? 512 : kTileThreads);
}

// One workgroup per block of a (batch of) image(s).
template <int N, int TV, bool SEPB, bool SYM = false>
__global__ void __launch_bounds__((tile_nt<N, 1>())) k_tile_corr_one(TileArgs a) {
  extern __shared__ cx<float> lds_t[];
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  const int ntile = a.tx * a.ty;
  corr_block_one<N, TV, SEPB, false, tile_nt<N, 1>(), SYM>(a, lb / ntile, lb % ntile, lds_t);
}
template <int N, bool SYM = false, bool Y2 = false>
__global__ void __launch_bounds__(2 * kTileThreads) k_tile_corr_pair(TileArgs a) {
  extern __shared__ cx<float> lds_t[];
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  const int ntile = a.tx * a.ty;
  corr_block_pair<N, false, SYM, Y2>(a, lb / ntile, lb % ntile, lds_t);
}

// Component stacks for matching: block `lb` of one image writes G_c(p) * scale, c < U, to
// plane c of a.stack (interleaved re, im; planes of ny nx pixels, so the stores of one
// component fill whole rows while the block is processed).
template <int N, int TV, bool SEPB, bool SYM = false>
__global__ void __launch_bounds__((tile_nt<N, 1>())) k_tile_stack_one(TileArgs a) {
  extern __shared__ cx<float> lds_t[];
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  corr_block_one<N, TV, SEPB, true, tile_nt<N, 1>(), SYM>(a, 0, a.tile0 + lb, lds_t);
}
template <int N, bool SYM = false>
__global__ void __launch_bounds__(2 * kTileThreads) k_tile_stack_pair(TileArgs a) {
  extern __shared__ cx<float> lds_t[];
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  corr_block_pair<N, true, SYM>(a, 0, a.tile0 + lb, lds_t);
}

// Batches of independent instances (every instance one image); item = (descriptor
// index, block index). Every launch holds the instances of one block shape and one form
// (plain or symmetric), so each kernel inlines a single block routine.
template <int N, int TV>
constexpr bool tile_sym_form() {
  return (N == 96 && TV == 64) || N == 128;
}

// tid >= 0: the thread index, passed in (see the persistent form)
template <int N, int TV, bool SEPB, int HV, bool SYM>
__device__ __forceinline__ void batch_block(const TileArgs& a, int blk, cx<float>* lds, int tid = -1) {
  if constexpr (HV == 2) corr_block_pair<N, false, SYM>(a, 0, blk, lds, tid);
  else corr_block_one<N, TV, SEPB, false, tile_nt<N, 1>(), SYM>(a, 0, blk, lds, tid);
}

// Item-table form: workgroup b runs item b. The host orders the items by decreasing
// cost, so the hardware dispatcher, which starts workgroups in order as CUs free up,
// schedules them longest first.
template <int N, int TV, bool SEPB, int HV, bool SYM>
__global__ void __launch_bounds__((tile_nt<N, HV>())) k_tile_items(const TileArgs* __restrict__ descs,
                                                                 const int2* __restrict__ items) {
  extern __shared__ cx<float> lds_t[];
  const int2 it = items[blockIdx.x];
  batch_block<N, TV, SEPB, HV, SYM>(descs[it.x], it.y, lds_t);
}

// Persistent form: a grid of resident workgroups takes the items (ordered by decreasing
// cost) one at a time from the counter ctr[0]. A workgroup that draws past the end counts
// itself out in ctr[1]; the last one to do so sets both counters back to zero, so the next
// launch (stream order) starts from a clean state without a separate clearing step.
template <int N, int TV, bool SEPB, int HV, bool SYM>
__global__ void __launch_bounds__((tile_nt<N, HV>())) k_tile_batch(const TileArgs* __restrict__ descs,
                                                                 const int2* __restrict__ items,
                                                                 int nitems, int* __restrict__ ctr) {
  extern __shared__ cx<float> lds_t[];
  int* slot = reinterpret_cast<int*>(lds_t);
  for (;;) {
    __syncthreads();   // the previous block has finished with the LDS
    if (threadIdx.x == 0) *slot = atomicAdd(&ctr[0], 1);
    __syncthreads();
    const int i = __builtin_amdgcn_readfirstlane(*slot);
    __syncthreads();   // every thread has read the slot before the block reuses the LDS
    if (i >= nitems) break;
    const int2 it = items[i];
    // the thread index through an empty asm statement: what the block routine derives
    // from it (twiddles in registers, addresses) is then recomputed for every block
    // instead of being hoisted out of the loop and held live across it
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    batch_block<N, TV, SEPB, HV, SYM>(descs[it.x], it.y, lds_t, tid);
  }
  if (threadIdx.x == 0 && atomicAdd(&ctr[1], 1) == (int)gridDim.x - 1) {
    atomicExch(&ctr[0], 0);
    atomicExch(&ctr[1], 0);
  }
}

// LDS of a launch: HV = 1: one image (+ the separate row buffer); HV = 2: the pair
// kernel's two images.
template <int N, int TV, bool SEPB, int HV>
constexpr size_t tile_lds() {
  return HV == 2 ? (size_t)2 * N * (N + 1) * sizeof(cx<float>)
                 : (size_t)(SEPB ? N + TV : N) * (N + 1) * sizeof(cx<float>);
}

template <int N, int TV, bool SEPB, int HV>
hipError_t launch_tile_kernel(hipStream_t s, unsigned nblk, const TileArgs& a, bool sym) {
  if constexpr (HV == 2) {
    static_assert(TV == 64, "the pair kernel has 64 x 64 blocks");
    constexpr size_t lds = tile_lds<N, TV, SEPB, HV>();
    const dim3 g(nblk), b(2 * kTileThreads);
    if constexpr (N == 96) {
      if (sym) {
        if (a.y2) hipLaunchKernelGGL((k_tile_corr_pair<N, true, true>), g, b, lds, s, a);
        else hipLaunchKernelGGL((k_tile_corr_pair<N, true>), g, b, lds, s, a);
        return last();
      }
    }
    if (a.y2) hipLaunchKernelGGL((k_tile_corr_pair<N, false, true>), g, b, lds, s, a);
    else hipLaunchKernelGGL((k_tile_corr_pair<N>), g, b, lds, s, a);
  } else {
    if (a.y2) return hipErrorInvalidValue;   // the one-group form has no second output
    if constexpr (N == 128 && !SEPB) {
      if (sym) {
        hipLaunchKernelGGL((k_tile_corr_one<N, TV, SEPB, true>), dim3(nblk), dim3(tile_nt<N, 1>()),
                           (tile_lds<N, TV, SEPB, HV>()), s, a);
        return last();
      }
    }
    hipLaunchKernelGGL((k_tile_corr_one<N, TV, SEPB>), dim3(nblk), dim3(tile_nt<N, 1>()),
                       (tile_lds<N, TV, SEPB, HV>()), s, a);
  }
  return last();
}

template <int N, int TV, bool SEPB, int HV>
hipError_t launch_stack_kernel(hipStream_t s, unsigned nblk, const TileArgs& a, bool sym) {
  if constexpr (HV == 2) {
    if constexpr (N == 96) {
      if (sym) {
        hipLaunchKernelGGL((k_tile_stack_pair<N, true>), dim3(nblk), dim3(2 * kTileThreads),
                           (tile_lds<N, TV, SEPB, HV>()), s, a);
        return last();
      }
    }
    if (sym) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_tile_stack_pair<N>), dim3(nblk), dim3(2 * kTileThreads),
                       (tile_lds<N, TV, SEPB, HV>()), s, a);
  } else {
    if constexpr (N == 128 && !SEPB) {
      if (sym) {
        hipLaunchKernelGGL((k_tile_stack_one<N, TV, SEPB, true>), dim3(nblk), dim3(tile_nt<N, 1>()),
                           (tile_lds<N, TV, SEPB, HV>()), s, a);
        return last();
      }
    }
    if (sym) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_tile_stack_one<N, TV, SEPB>), dim3(nblk), dim3(tile_nt<N, 1>()),
                       (tile_lds<N, TV, SEPB, HV>()), s, a);
  }
  return last();
}

template <int N, int TV, bool SEPB, int HV>
hipError_t prepare_tile_kernel() {
  hipError_t e = allow_lds(k_tile_batch<N, TV, SEPB, HV, false>);
  if (e == hipSuccess) e = allow_lds(k_tile_items<N, TV, SEPB, HV, false>);
  if constexpr (tile_sym_form<N, TV>()) {
    if (e == hipSuccess) e = allow_lds(k_tile_batch<N, TV, SEPB, HV, true>);
    if (e == hipSuccess) e = allow_lds(k_tile_items<N, TV, SEPB, HV, true>);
  }
  if (e == hipSuccess) {
    if constexpr (HV == 2) {
      e = allow_lds(k_tile_stack_pair<N>);
      if constexpr (N == 96) {
        if (e == hipSuccess) e = allow_lds(k_tile_stack_pair<N, true>);
      }
    } else {
      e = allow_lds(k_tile_stack_one<N, TV, SEPB>);
      if constexpr (N == 128 && !SEPB) {
        if (e == hipSuccess) e = allow_lds(k_tile_stack_one<N, TV, SEPB, true>);
      }
    }
  }
  if (e != hipSuccess) return e;
  if constexpr (HV == 2) {
    e = allow_lds(k_tile_corr_pair<N>);
    if (e == hipSuccess) e = allow_lds(k_tile_corr_pair<N, false, true>);
    if constexpr (N == 96) {
      if (e == hipSuccess) e = allow_lds(k_tile_corr_pair<N, true>);
      if (e == hipSuccess) e = allow_lds(k_tile_corr_pair<N, true, true>);
    }
    return e;
  } else {
    e = allow_lds(k_tile_corr_one<N, TV, SEPB>);
    if constexpr (N == 128 && !SEPB) {
      if (e == hipSuccess) e = allow_lds(k_tile_corr_one<N, TV, SEPB, true>);
    }
    return e;
  }
}

}  // namespace

// (N, TV, separate row buffer, 1 = one group per component / 2 = component pairs)
#define ECC_TILE_CONFIGS(X) \
  X(64, 64, true, 2) X(96, 64, false, 2) X(128, 64, false, 1) X(128, 96, false, 1)

bool tile_supported(int N, int TV) {
#define ECC_TS(n, tv, sb, hv) if (N == n && TV == tv) return true;
  ECC_TILE_CONFIGS(ECC_TS)
#undef ECC_TS
  return false;
}

size_t tile_lds_bytes(int N, int TV) {
#define ECC_TB(n, tv, sb, hv) if (N == n && TV == tv) return tile_lds<n, tv, sb, hv>();
  ECC_TILE_CONFIGS(ECC_TB)
#undef ECC_TB
  return 0;
}

hipError_t launch_tile_corr(hipStream_t s, int N, int TV, int batch, const float* H, long long planeH,
                            int ldH, const Field& fld, float* y, long long planeY, int ldY, int ny,
                            int nx, int R, int T, int U, int kofs, const float* w, float scale,
                            const cx<float>* Fs, bool sym, float* y2, const float* mulsig,
                            long long planeMul, int ldMul) {
  if (T < 1 || T > TV || T > N - 2 * R) return hipErrorInvalidValue;
  if (sym && (!tile_symmetric(N, TV) || kofs != 0)) return hipErrorInvalidValue;
  if (y2 && (!tile_has_y2(N, TV) || !mulsig)) return hipErrorInvalidValue;
  TileArgs a{};
  a.H = H;
  a.planeH = planeH;
  a.ldH = ldH;
  a.fld = fld;
  a.y = y;
  a.planeY = planeY;
  a.ldY = ldY;
  a.ny = ny;
  a.nx = nx;
  a.R = R;
  a.T = T;
  a.tx = (nx + T - 1) / T;
  a.ty = (ny + T - 1) / T;
  a.U = U;
  a.kofs = kofs;
  a.w = w;
  a.scale = scale;
  a.Fs = Fs;
  a.y2 = y2;
  a.mulsig = mulsig;
  a.planeMul = planeMul;
  a.ldMul = ldMul;
  const long long nblk = (long long)a.tx * a.ty * batch;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
#define ECC_TL(n, tv, sb, hv) \
  if (N == n && TV == tv) return launch_tile_kernel<n, tv, sb, hv>(s, (unsigned)nblk, a, sym);
  ECC_TILE_CONFIGS(ECC_TL)
#undef ECC_TL
  return hipErrorInvalidValue;
}

bool tile_symmetric(int N, int TV) {
#define ECC_TSY(n, tv, sb, hv) if (N == n && TV == tv) return tile_sym_form<n, tv>();
  ECC_TILE_CONFIGS(ECC_TSY)
#undef ECC_TSY
  return false;
}
bool tile_has_y2(int N, int TV) {
#define ECC_TY(n, tv, sb, hv) if (N == n && TV == tv) return hv == 2;
  ECC_TILE_CONFIGS(ECC_TY)
#undef ECC_TY
  return false;
}

hipError_t launch_tile_stack(hipStream_t s, int N, int TV, const float* H, int ldH, int ny, int nx, int R,
                             int T, int U, float scale, const cx<float>* Fs, float* stack, bool sym, int by0,
                             int by1) {
  if (T < 1 || T > TV || T > N - 2 * R) return hipErrorInvalidValue;
  const int nby = (ny + T - 1) / T;
  if (by1 < 0) by1 = nby;
  if (by0 < 0 || by1 > nby || by0 >= by1) return hipErrorInvalidValue;
  if (sym && !tile_symmetric(N, TV)) return hipErrorInvalidValue;
  TileArgs a{};
  a.H = H;
  a.ldH = ldH;
  a.ny = ny;
  a.nx = nx;
  a.R = R;
  a.T = T;
  a.tx = (nx + T - 1) / T;
  a.ty = (ny + T - 1) / T;
  a.U = U;
  a.scale = scale;
  a.Fs = Fs;
  a.stack = stack;
  a.stack_y0 = by0 * T;
  a.stack_plane = stack_pitch((long long)((ny < by1 * T ? ny : by1 * T) - a.stack_y0) * nx);
  a.tile0 = by0 * a.tx;
  const long long nblk = (long long)a.tx * (by1 - by0);
#define ECC_TSK(n, tv, sb, hv) \
  if (N == n && TV == tv) return launch_stack_kernel<n, tv, sb, hv>(s, (unsigned)nblk, a, sym);
  ECC_TILE_CONFIGS(ECC_TSK)
#undef ECC_TSK
  return hipErrorInvalidValue;
}

int tile_threads(int N, int TV) {
#define ECC_TT(n, tv, sb, hv) if (N == n && TV == tv) return tile_nt<n, hv>();
  ECC_TILE_CONFIGS(ECC_TT)
#undef ECC_TT
  return 0;
}

int tile_blocks_per_cu(int N, int TV) {
  int nb = 0;
#define ECC_TO(n, tv, sb, hv)                                                                   \
  if (N == n && TV == tv) {                                                                     \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tile_items<n, tv, sb, hv, false>,   \
                                                     tile_nt<n, hv>(),                         \
                                                     tile_lds<n, tv, sb, hv>()) != hipSuccess)  \
      nb = 1;                                                                                   \
    return nb > 0 ? nb : 1;                                                                     \
  }
  ECC_TILE_CONFIGS(ECC_TO)
#undef ECC_TO
  return 1;
}

template <int N, int TV, bool SEPB, int HV, bool SYM>
hipError_t launch_batch_kernel(hipStream_t s, int nwg, const TileArgs* descs, const int2* items, int nitems,
                               int* ctr) {
  constexpr size_t lds = tile_lds<N, TV, SEPB, HV>();
  if (ctr == nullptr)
    hipLaunchKernelGGL((k_tile_items<N, TV, SEPB, HV, SYM>), dim3(nwg), dim3(tile_nt<N, HV>()), lds, s, descs,
                       items);
  else
    hipLaunchKernelGGL((k_tile_batch<N, TV, SEPB, HV, SYM>), dim3(nwg), dim3(tile_nt<N, HV>()), lds, s, descs,
                       items, nitems, ctr);
  return last();
}

template <int N, int TV, bool SEPB, int HV>
hipError_t launch_batch_form(hipStream_t s, bool sym, int nwg, const TileArgs* descs, const int2* items,
                             int nitems, int* ctr) {
  if constexpr (tile_sym_form<N, TV>()) {
    if (sym) return launch_batch_kernel<N, TV, SEPB, HV, true>(s, nwg, descs, items, nitems, ctr);
  }
  if (sym) return hipErrorInvalidValue;
  return launch_batch_kernel<N, TV, SEPB, HV, false>(s, nwg, descs, items, nitems, ctr);
}

hipError_t launch_tile_batch(hipStream_t s, int N, int TV, bool sym, int nwg, const TileArgs* descs,
                             const int2* items, int nitems, int* ctr) {
  if (nwg < 1 || nitems < 1 || (ctr == nullptr && nwg != nitems)) return hipErrorInvalidValue;
#define ECC_TBL(n, tv, sb, hv) \
  if (N == n && TV == tv) return launch_batch_form<n, tv, sb, hv>(s, sym, nwg, descs, items, nitems, ctr);
  ECC_TILE_CONFIGS(ECC_TBL)
#undef ECC_TBL
  return hipErrorInvalidValue;
}

hipError_t prepare_tile_kernels() {
  hipError_t e = hipSuccess;
#define ECC_TP(n, tv, sb, hv) \
  if (e == hipSuccess) e = prepare_tile_kernel<n, tv, sb, hv>();
  ECC_TILE_CONFIGS(ECC_TP)
#undef ECC_TP
  return e;
}

}  // namespace ecc
