// Launch interface between the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_device.hpp"

namespace ecc {

// Transform-set geometry chosen on the host for one kernel launch.
struct RowCfg {   // blocked layout: B transforms (rows) per workgroup, TF threads each
  int B, TF, NB, EPX;
};
struct ColCfg {   // interleaved layout: B = 2^lgB adjacent columns per workgroup
  int lgB, nthr, NB, EPT;
};

struct Field {    // per-pixel angle alpha(q) = mul * g(field(q)) + add, g = id or ln
  const float* ptr;
  long long plane;
  int ld;
  int log_mode;
  double mul, add;
};

// ---- correlation path
hipError_t launch_rows_r2c(hipStream_t s, const RowCfg& c, int batch, const float* H, long long planeH,
                           int ldH, cx<float>* A, long long planeA, int ldA, int ny, int nx, int W,
                           const FftDesc& d, const cx<float>* tw);
hipError_t launch_cols_fwd(hipStream_t s, const ColCfg& c, int batch, const cx<float>* A,
                           long long planeA, int ldA, int nyValid, int ncols, cx<float>* out,
                           long long planeOut, int ldOut, const FftDesc& d, const cx<float>* tw);
hipError_t launch_corr_cols(hipStream_t s, const ColCfg& c, int batch, int kchunk,
                            const cx<float>* Hh, long long planeHh, int ldHh, const cx<float>* Fh,
                            long long planeFk, int ldF, int fullplane, const float* parity,
                            cx<float>* T, long long planeTk, long long planeTimg, int ldT, int ny,
                            int Px, int W, int U, int conj_mode, const FftDesc& d,
                            const cx<float>* tw);
hipError_t launch_corr_rows(hipStream_t s, const RowCfg& c, int batch, const cx<float>* T,
                            long long planeTk, long long planeTimg, int ldT, const Field& fld,
                            float* y, long long planeY, int ldY, int ny, int nx, int U,
                            const float* w, float scale, float* y2, const float* mulsig,
                            long long planeMul, int ldMul, float y2scale, int kofs, int accum,
                            const FftDesc& d, const cx<float>* tw);
hipError_t launch_match_rows(hipStream_t s, const RowCfg& c, const cx<float>* T, long long planeTk,
                             int ldT, float* score, int* index, int ldOut, int ny, int nx, int U,
                             const float* w, float scale, int n_angles, const float* angle_tab,
                             const FftDesc& d, const cx<float>* tw);

// joint rotation and scale fields: angle theta(q) and scale s(q) of every pixel
struct JointField {
  const float* theta;
  long long plane_t;
  int ld_t;
  const float* scale;
  long long plane_s;
  int ld_s;
  double om1;   // omega_1 = 2 pi / L of the log-radial modes
};

// ---- convolution path
hipError_t launch_conv_rows_fwd(hipStream_t s, const RowCfg& c, int batch, const float* H,
                                long long planeH, int ldH, const Field& fld, int sig_norm,
                                int nsig, cx<float>* Bk, long long planeBk, long long planeBsig,
                                long long planeBimg, int ldB, int ny, int nx, int U,
                                const FftDesc& d, const cx<float>* tw);
// the same for joint plans (components in the half-set order k = 0: l = 0..h; k = 1..K:
// l = -h..h; n = 2h + 1 log-radial modes)
hipError_t launch_conv_rows_fwd_joint(hipStream_t s, const RowCfg& c, int batch, const float* H, long long planeH,
                                      int ldH, const JointField& jf, int sig_norm, int nsig, cx<float>* Bk,
                                      long long planeBk, long long planeBsig, long long planeBimg, int ldB, int ny,
                                      int nx, int U, int n, const FftDesc& d, const cx<float>* tw);
// joint plan components (float64): f_tmp (n + 2) x (2K + 1), c_tmp (2K + 1) x n, comps U x S x S
hipError_t launch_joint_components(hipStream_t s, const float* F, int S, int K, int M, int n, double u_lo,
                                   double u_hi, double L, cx<double>* f_tmp, cx<double>* c_tmp, cx<double>* comps);
// groups > 1: the components are split into that many consecutive groups (more
// workgroups for small batches), each summed in order into a Py x Px partial plane per
// image and signal in `part` (groups x batch x nsig planes), then the partial planes are
// added in group order before the inverse transform.
hipError_t launch_conv_cols(hipStream_t s, const ColCfg& c, int batch, const cx<float>* Bk,
                            long long planeBk, long long planeBsig, long long planeBimg, int ldB,
                            const cx<float>* Fh, long long planeFk, int ldF, int fullplane,
                            const float* parity, const float* w, cx<float>* C, long long planeCsig,
                            long long planeCimg, int ldC, int ny, int Py, int Px, int W, int U,
                            int nsig, const FftDesc& d, const cx<float>* tw, int groups = 1,
                            cx<float>* part = nullptr);
hipError_t launch_conv_rows_inv(hipStream_t s, const RowCfg& c, int batch, const cx<float>* C,
                                long long planeCsig, long long planeCimg, int ldC, float* y,
                                long long planeY, int ldY, int ny, int nx, int nsig, float scale,
                                const FftDesc& d, const cx<float>* tw);

// ---- generic complex transforms (float or double), used by plans and the adjoint
template <typename T>
hipError_t launch_fft_rows(hipStream_t s, const RowCfg& c, int nplanes, int dir, const cx<T>* in,
                           long long planeIn, int ldIn, int nrows, int nvalid, int shift_in,
                           cx<T>* out, long long planeOut, int ldOut, int nstore, int shift_out,
                           const FftDesc& d, const cx<T>* tw);
// mul != NULL: every input element is multiplied on load by mul[j ldIn + v] (the same
// multiplier plane for every input plane)
template <typename T>
hipError_t launch_fft_cols(hipStream_t s, const ColCfg& c, int nplanes, int dir, const cx<T>* in,
                           long long planeIn, int ldIn, int ncols, int nvalid, int shift_in,
                           cx<T>* out, long long planeOut, int ldOut, int nstore, int shift_out,
                           const FftDesc& d, const cx<T>* tw, const cx<T>* mul = nullptr);

// ---- filter plans (float64)
hipError_t launch_polar_dft(hipStream_t s, const float* F, int S, int K, int M, const int* d2list,
                            int nrad, cx<double>* fk);
hipError_t launch_synth_rotation(hipStream_t s, const float* F, int S, int K, const int* rmap,
                                 const cx<double>* fk, cx<double>* comps);
hipError_t launch_scale_components(hipStream_t s, double sigma0, double u_lo, double u_hi,
                                   double L, int n, int R, cx<double>* comps);
hipError_t launch_d2f(hipStream_t s, const cx<double>* in, cx<float>* out, long long n);
hipError_t launch_conj_d(hipStream_t s, const cx<double>* in, cx<double>* out, long long n);   // out = conj(in)
hipError_t launch_f2d(hipStream_t s, const cx<float>* in, cx<double>* out, long long n);
hipError_t launch_scale_f(hipStream_t s, float* y, long long n, float a);                      // y *= a

// ---- adjoint helpers
hipError_t launch_grad_filter_cols(hipStream_t s, const ColCfg& c, int batch,
                                   const cx<float>* Bk, long long planeBk, long long planeBimg,
                                   int ldB, const cx<float>* Gh, long long planeGimg, int ldG,
                                   cx<float>* D, long long planeDk, int ldD, int ny, int Py, int Px,
                                   int U, const FftDesc& d, const cx<float>* tw);
hipError_t launch_grad_filter_finish(hipStream_t s, const cx<float>* win, long long planeWin,
                                     int ldWin, const float* w, float scale, cx<float>* out, int S,
                                     int U);

// ---- correlation row kernel for transform lengths with a compiled schedule P = R0 R1 R2
bool fixed_split(int P, int* R0, int* R1, int* R2);
hipError_t launch_corr_rows_fixed(hipStream_t s, int NR, int batch, const cx<float>* T, long long planeTk,
                                  long long planeTimg, int ldT, const Field& fld, float* y,
                                  long long planeY, int ldY, int ny, int nx, int U, const float* w,
                                  float scale_, float* y2, const float* mulsig, long long planeMul,
                                  int ldMul, float y2scale, int kofs, int accum, int Px,
                                  const cx<float>* tw);

// ---- tiled (overlap-save) correlation: one workgroup per T x T output block, N x N
// transforms on chip (N = 64, 96, 128; TV = 64 or 96 bounds T)
struct TileArgs {          // one correlation job (batch of images of one shape)
  const float* H;
  long long planeH;
  int ldH;
  Field fld;
  float* y;
  long long planeY;
  int ldY;
  int ny, nx, R, T, tx, ty, U, kofs;   // tx, ty: blocks across and down
  const float* w;
  float scale;
  const cx<float>* Fs;     // U block spectra of N x N
  float* stack;            // component stacks (matching): U planes (re, im), or NULL
  long long stack_plane;   // complex values from one stack plane to the next (stack_pitch)
  int stack_y0;            // first image row held by the stack
  int tile0;               // stack kernels: block index of the launch's first workgroup
  // second output (adjoint w.r.t. the field): y2 = scale * mulsig * sum_c w_c (kofs + c)
  // Im(e^{i (kofs + c) alpha} G_c), or NULL
  float* y2;
  const float* mulsig;
  long long planeMul;
  int ldMul;
  int sym;                 // batch descriptors: the symmetric pair form (centred spectra)
};
bool tile_supported(int N, int TV);
// block shapes with the symmetric pair form (rotation filters: centred block spectra with
// F~_c(-w) = (-1)^c F~_c(w), component offset 0)
bool tile_symmetric(int N, int TV);
size_t tile_lds_bytes(int N, int TV);
int tile_threads(int N, int TV);
// Plane pitch (complex values) of a component stack of npix pixels: the planes start on
// 512-byte boundaries, 1 KiB past a multiple of 512 bytes beyond the plane, so that the U
// planes an angle search reads side by side are not a power of two apart in memory (at
// 1024 x 1024 they would be 2^23 bytes apart, and the reads ran 13% slower).
inline long long stack_pitch(long long npix) { return (npix + 63) / 64 * 64 + 128; }
// component stack of the block rows [by0, by1) of one image (by1 < 0: to the last):
// with y0 = by0 T, rows = min(ny, by1 T) - y0 and P = stack_pitch(rows nx),
// stack[2 (c P + (y - y0) nx + x) .. +1] = G_c(y, x) * scale for y0 <= y < y0 + rows
hipError_t launch_tile_stack(hipStream_t s, int N, int TV, const float* H, int ldH, int ny, int nx, int R,
                             int T, int U, float scale, const cx<float>* Fs, float* stack, bool sym = false,
                             int by0 = 0, int by1 = -1);
// angle search over a component stack of npix pixels (planes stack_pitch(npix) apart):
// score = max_m sum_c Re(e^{2 pi i c m / A} w_c G_c),
// index = first maximising m; prec 0 = float32 FMA, 1 = float16 hi/lo MFMA, 2 = bfloat16
// hi/lo MFMA. dtab: float32 [64][64] (angle m, stack entry k) = w_{k/2} cos / -w_{k/2} sin.
hipError_t launch_match_angles(hipStream_t s, int prec, const float* stack, int U, long long npix, int A,
                               const float* dtab, float* score, int* index, int ldOut, int nx);
int tile_blocks_per_cu(int N, int TV);   // resident workgroups per CU (occupancy query)
// batches: item = (descriptor index, block index), all of one block shape and one form
// (sym: the symmetric form, centred spectra). Item-table form (ctr == NULL): nwg = nitems
// workgroups, workgroup b runs item b. Persistent form: nwg workgroups take the items in
// order from the counter pair ctr[0..1], which must be zero at launch and is zero again
// when the launch ends; launches sharing one counter pair must not overlap.
hipError_t launch_tile_batch(hipStream_t s, int N, int TV, bool sym, int nwg, const TileArgs* descs,
                             const int2* items, int nitems, int* ctr);
hipError_t launch_tile_corr(hipStream_t s, int N, int TV, int batch, const float* H, long long planeH,
                            int ldH, const Field& fld, float* y, long long planeY, int ldY, int ny,
                            int nx, int R, int T, int U, int kofs, const float* w, float scale,
                            const cx<float>* Fs, bool sym = false, float* y2 = nullptr,
                            const float* mulsig = nullptr, long long planeMul = 0, int ldMul = 0);
// block shapes whose correlation kernel can also write the second (y2) output
bool tile_has_y2(int N, int TV);

// ---- tiled (overlap-save) convolution: one workgroup (256 threads) per T x T block
// Block spectra of the tiled convolution: per component a plane of N rows of pitch N + 1
// complex64 values, the plane rounded up to a multiple of 128 values (1 KB), so that a
// plane can be copied into LDS in whole 1 KB pieces with the odd pitch kept.
constexpr int tconv_pitch(int N) { return N + 1; }
constexpr int tconv_plane(int N) { return (N * (N + 1) + 127) / 128 * 128; }

struct TileConvArgs {
  const float* H;
  long long planeH;
  int ldH;
  Field fld;               // phase e^{-i c alpha}
  int sig_norm;            // signal divided by field^2
  int nsig;                // 1: y = scale Re sum; 2: ratio of the sums for H/f^2 and 1/f^2
  int step;                // set by the launcher: 0 plain, 1 numerator, 2 denominator
  float* y;
  long long planeY;
  int ldY;
  int ny, nx, R, T, tx, ty, U;   // tx, ty set by the launcher
  const float* w;
  float scale;
  const cx<float>* Fs;     // U block spectra (tconv_plane(N) values apart, pitch N + 1),
                           // F_c at (x - R) mod N
  // joint rotation and scale plans (joint_n > 0: n log-radial modes, angular frequencies
  // 0..joint_K): the phase is e^{-i (k alpha + omega_l ln s)} with alpha from fld (radians)
  // and s from jscale, omega_l = l joint_om1; the signal is divided by s^2 when sig_norm
  int joint_n, joint_K;
  float joint_om1;
  const float* jscale;
  long long plane_s;
  int ld_s;
};
// Filter part of the convolution adjoint on chip (section 4 adjoint of the extended
// convolution): per block of outputs and component k, the lags x in [-R, R]^2 of
// sum_{p in block} g(p) conj(M_k(p - x)), M_k = H e^{-ik theta}, written as partial sums
// part[block][k][R + x_y][R + x_x] (complex, unnormalised: times 1 / N^2).
struct TileGradFArgs {
  const float* H;          // signal
  long long planeH;
  int ldH;
  Field fld;               // phase e^{-i k alpha}
  const float* G;          // gradient of the output
  long long planeG;
  int ldG;
  cx<float>* part;         // blocks x U x S x S
  int ny, nx, R, T, tx, ty, U;
};
bool tgradf_supported(int N, int TV);
hipError_t launch_tile_gradf(hipStream_t s, int N, int TV, int batch, const TileGradFArgs& a);
// out[k][a][b] = w_k * scale * sum over nblk blocks of part[block][k][a][b] (order fixed:
// 64 chunks of consecutive blocks, each summed in block order, then the chunks in order;
// float64 sums); scratch: gradf_reduce_scratch(U, S) bytes of device memory
size_t gradf_reduce_scratch(int U, int S);
hipError_t launch_gradf_reduce(hipStream_t s, const cx<float>* part, int nblk, int U, int S, const float* w,
                               float scale, cx<float>* out, void* scratch);
// ---- normalised convolution by overlap-add blocks: num + i den of two signals sharing
// the field in one launch (sources T x T per block, regions of N x N, N >= T + 2R, added
// in a fixed order by a second kernel that also divides)
struct TileRatioArgs {
  const float* H;
  long long planeH;
  int ldH;
  Field fld;               // phase e^{-i c alpha}
  int sig_norm;            // 1: s1 = H / f^2, s2 = 1 / f^2; 0: s1 = H, s2 = 1
  float* y;
  long long planeY;
  int ldY;
  int ny, nx, R, T, tx, ty, U;   // tx, ty set by the launcher
  const float2* Fs;        // U planes of N x N (w_c rho_a, w_c rho_b), [column freq][row freq]
  const float* par;        // parity p_c of each component (+1: real spectra, -1: imaginary)
  cx<float>* part;         // partial sums: blocks x N x N (tratio_scratch_bytes)
};
bool tratio_supported(int N, int TV);
size_t tratio_scratch_bytes(int N, int T, int batch, int ny, int nx);
// prec 0: float32; 1 / 2: the radix-16 passes of the forward transforms on the matrix
// cores with float16 / bfloat16 hi + lo operands (float32 accumulation). plain (prec 0
// only): the extended convolution of the one signal s1 instead of the ratio,
// y = Re sum_c w_c (s1 e^{-i c alpha}) * F_c, one forward transform per component
hipError_t launch_tile_ratio(hipStream_t s, int N, int TV, int batch, const TileRatioArgs& a, int prec = 0,
                             bool plain = false);
// spectra of the overlap-add ratio kernel from the centred float64 spectra of the
// components (U planes of N x N, [row freq][column freq]): per component the real parts of
// the spectra of Re F_c and Im F_c (parity +1) or their imaginary parts (parity -1), times
// w_c, as float2 planes [column freq][row freq]
hipError_t launch_ratio_spectra(hipStream_t s, const cx<double>* spec, int U, int N, const float* w,
                                const float* par, float2* out);
bool tconv_supported(int N, int TV);
size_t tconv_lds_bytes(int N);
hipError_t launch_tile_conv(hipStream_t s, int N, int TV, int batch, const TileConvArgs& a);
// Direct (spatial) extended correlation or convolution (conv) for filter sides S in
// {3, 5, ..., 15}: the fields of TileArgs as for launch_tile_corr's single form (H, planeH,
// ldH, fld, y, planeY, ldY, ny, nx, R = (S - 1) / 2, U, kofs (0 for the convolution), w,
// scale), Fs = the U components as U x S x S complex64 values; blocks of 16 x 64 outputs
// (tx, ty set by the launcher, or by direct_blocks for batch descriptors).
bool direct_supported(int S);
void direct_blocks(int ny, int nx, int* tx, int* ty);
hipError_t launch_direct(hipStream_t s, bool conv, int S, int batch, const TileArgs& a);
hipError_t launch_direct_items(hipStream_t s, bool conv, int S, const TileArgs* descs, const int2* items,
                               int nitems);
// Batches of convolutions: one workgroup per item (descriptor index, block index) of
// device descriptors (plain form: nsig = 1, step = 0, tx and ty set) and items.
hipError_t launch_tile_conv_items(hipStream_t s, int N, int TV, const TileConvArgs* descs, const int2* items,
                                  int nitems);

// LDS needed for a launch, in bytes (twiddles + transform buffers).
size_t lds_rows(const RowCfg& c, const FftDesc& d, size_t elem);
size_t lds_cols(const ColCfg& c, const FftDesc& d, size_t elem);
hipError_t prepare_kernels();   // raises per-kernel dynamic LDS limits once

// ---- steering in 3D (volumes [z][y][x]; spherical-harmonic components, Wigner-D)
constexpr int kMaxSteerK = 8;
// A[ri][i][m] = sum_j F(r w_ij) e^{-i m phi_j}, m = 0..K, r = sqrt(d2[ri]), polar nodes
// gl_t (cos theta), M azimuths; float64, F trilinear (zero outside the S^3 array)
hipError_t launch_sh_azimuth(hipStream_t s, const float* F, int S, int K, int M, int nt, const double* gl_t, int nr,
                             const int* d2, cx<double>* A);
// f[ri][l][m + K] = f_l^m(r) by the polar quadrature (weights gl_w)
hipError_t launch_sh_polar(hipStream_t s, const cx<double>* A, int nr, int nt, int K, int M, const double* gl_t,
                           const double* gl_w, cx<double>* f);
// comps[c][S^3] = f_l^m(|q|) Y_l^{m'}(q/|q|) for hs[c] = (l, m', m), rindex[d2] = ri
hipError_t launch_sh_components(hipStream_t s, const float* F, int S, int K, int U, const int4* hs,
                                const int* rindex, const cx<double>* f, cx<double>* comps);
hipError_t launch_real_to_cx(hipStream_t s, const float* in, cx<float>* out, long long n);
// Batched float32 transforms of length P with a compiled schedule (fx3_supported(P)), no
// circular shift: columns (16 adjacent per workgroup; mul as launch_fft_cols) and rows.
// tw: the transform's pass-1/pass-2 twiddle table (Transform::fx()).
bool fx3_supported(int P);
hipError_t launch_fx_cols(hipStream_t s, int P, int dir, int nplanes, const cx<float>* in, long long planeIn,
                          int ldIn, int ncols, int nvalid, cx<float>* out, long long planeOut, int ldOut,
                          int nstore, const cx<float>* tw, const cx<float>* mul);
hipError_t launch_fx_rows(hipStream_t s, int P, int dir, int nplanes, const cx<float>* in, long long planeIn,
                          int ldIn, int nrows, int nvalid, cx<float>* out, long long planeOut, int ldOut,
                          int nstore, const cx<float>* tw);
// Forward column transforms of nplanes planes summed with weights against as many
// spectra: out[i][v] = sum_u w_u Sp_u[i][v] DFT(in_u)[i][v], i < P (row pitch ldOut for
// Sp and out). The components are split into at most `groups` consecutive groups, summed
// in order within each group into planes of `part` (planePart apart; unused with one
// group), then the groups are added in order. S > 0: Sp holds partial spectra (each
// component transformed along the other two axes only: S = 2R + 1 planes, offset j - R in
// plane j), whose full column is formed on chip by the forward transform along this axis.
hipError_t launch_fx_cols_accum(hipStream_t s, int P, int nplanes, const cx<float>* in, long long planeIn, int ldIn,
                                int ncols, int nvalid, const cx<float>* Sp, long long planeSp, int S, int R,
                                const float* w, int groups, cx<float>* part, long long planePart, cx<float>* out,
                                int ldOut, const cx<float>* tw);
// The correlation's inverse pass along z with the product formed on chip: for component
// c < nplanes, out_c rows i < nstore = IDFT(DFT+(partial column of sp_c) * A) along the
// rows (partial spectra as above, transformed with direction +1; planeSp, planeOut apart;
// row pitch ld for sp, A and out).
hipError_t launch_fx_cols_corr(hipStream_t s, int P, int nplanes, const cx<float>* sp, long long planeSp, int ld,
                               int ncols, int S, int R, const cx<float>* A, cx<float>* out, long long planeOut,
                               int nstore, const cx<float>* tw);
// The correlation's last inverse pass (along x, compiled length P) fused with the Wigner-D
// combination: y[row][x] = scale sum_c w_c Re(D_c(x) IDFT(in_c[row])[x]) for K <= kFusedWignerK
// and nx <= 192; alpha, beta, gamma and y are nrows x nx.
constexpr int kFusedWignerK = 4;
bool fx_rows_wigner_supported(int P, int K, int nx);
hipError_t launch_fx_rows_wigner(hipStream_t s, int P, int K, const cx<float>* in, long long planeIn, int ldIn,
                                 int nrows, int nvalid, int nx, const float* alpha, const float* beta,
                                 const float* gamma, const double* coef, const float* w, float* y, float scale,
                                 const cx<float>* tw);
hipError_t prepare_fx_kernels();
// A[v] = sum_c w_c X[c][v] Sp[c][v]
hipError_t launch_spec_accumulate(hipStream_t s, const cx<float>* X, const cx<float>* Sp, const float* w, long long V,
                                  int U, cx<float>* A);
hipError_t launch_real_part(hipStream_t s, const cx<float>* in, float* y, long long n, float scale);
// mode 0: y[v] = scale sum_c w_c Re(D_c(v) G[c][v]); mode 1: M[c][v] = H[v] D_c(v); D_c the
// Wigner-D entry of half-set component c at the voxel's Euler angles; coef: Wigner's
// coefficients, one per term of d^l_{m'm}, in half-set order
hipError_t launch_wigner_voxels(hipStream_t s, int K, int mode, const float* alpha, const float* beta,
                                const float* gamma, long long nvox, const double* coef, const float* w,
                                const cx<float>* G, const float* H, float* y, cx<float>* M, float scale);

}  // namespace ecc
