// Internal declarations of libdlx: plan layout, kernel argument blocks and
// launcher prototypes. Not part of the public ABI (see include/dlx.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "dlx.h"

namespace dlx {

constexpr double kTwoPi = 6.283185307179586476925286766559;

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Per-wavelength constants, read by the kernels.
struct WlInfo {
  double lam;     // metres
  float w;        // spectral weight
  float scale;    // dx * du / lambda, the focal-field factor
  float kphase;   // 2 pi / lambda
  float pad;
};

// A planar complex operand. FP32: re plane at base, im plane at base + plane
// (floats). Split BF16: four planes re hi, re lo, im hi, im lo, `plane`
// 16-bit elements apart. The item's matrix starts at
// base + (psf % L) * by_wl + local_psf * by_psf; rows are `ld` elements
// apart (ld a multiple of 16; padded columns are never read: the loaders
// mask k >= K). All offsets are in elements of the operand's type.
struct Operand {
  const void* base;
  long long plane;
  long long by_wl;
  long long by_psf;
  int ld;
};

// The matrix-Fourier stages of one forward+gradient evaluation.
//   F1  T = M_l P              (pupil field generated in the operand loader)
//   F2  E = c T M_l^T          stored FP32 (intensity, binning and the adjoint read it)
//   B3  U^T = conj(M_l)^T Y^T  stored; the seed Y = w phi G E is formed in the operand loader
//                              from E and the frame's seed weights G = K flat r
//   B4  W = c M_l^H U          epilogue: g = 2 Im(conj(P) W) (2 pi / l) summed over a group; position partials
//
// Symmetric fold. On the pixel-centred grids the coordinates pair up, x[N-1-n] = -x[n], so the
// DFT matrix D[a][k] = Dr + i Di satisfies D[a][K-1-k] = conj(D[a][k]) = D[A-1-a][k]. A product
// sum_k D[a][k] X[k] then needs only the sums Xe[k] = X[k] + X[K-1-k] and differences
// Xo[k] = X[k] - X[K-1-k] for k < ceil(K/2):
//   P = sum Dr Xe,  R = sum Di Xo,   out[a] = P + i R,   out[A-1-a] = P - i R,
// four real products of half the depth over half the DFT rows: a quarter of the dense work.
// The data operands of the fold (pupil field, T, E, G, U^T) keep the lower half of each row in
// place and move the upper half to end at the leading dimension ld (column c >= ceil(N/2) at
// c + ld - N), so the mirror of the 16-byte chunk at k is the chunk at ld - 4 - k, reversed.
enum GemmKind { KIND_F1 = 0, KIND_F2 = 1, KIND_B3 = 3, KIND_B4 = 4 };

struct GemmArgs {
  int M, N, K;          // C[M][N] = sum_k A[i][k] B[j][k] per PSF
  int tiles_m, tiles_n;
  int n_items;          // PSFs (F1, F2, B3) or PSF groups (B4)
  int L, S;             // wavelengths, sources
  int psf0;             // global index of the chunk's first PSF
  int frame0;           // first frame of the chunk
  int group_size;       // PSFs per group item
  int groups;           // B4: groups in the chunk
  int n_chunk_psf;
  int conj_a, conj_b;
  int ksplit;           // B4: K range split over ksplit items (the epilogue is linear in W)
  Operand A, B;
  // pupil field pieces: P[m][n] = P0T[n][m] * ty[m] * tx[n] (F1 loader, B4 epilogue)
  const float* tx;
  const float* ty;
  long long tilt_plane;
  int ldt;
  const float* p0t;
  long long p0_plane;
  long long p0_by_wl;
  int ldp;
  const WlInfo* wl;
  const float* sources;   // [F][S][3]
  // B3: seed weights G of the chunk's frames [nf][No][ldg]
  const float* seedw;
  long long seedw_by_frame;
  // dense outputs (F1: T, F2: E, B3: U^T), indexed by local PSF; E is FP32, the others are
  // split BF16 under BF16X3 in the dense kernels and FP32 in the folded ones
  void* out;
  long long out_plane;
  long long out_by_psf;
  int ldo;
  // group partials: B4 dL/dOPD [groups][Ni*Ni]
  float* part;
  int accumulate;
  // per-(PSF, tile) FP64 partials: B4 positions [n_psf][tiles][2]
  double* red;
  const double* xcoord;   // pupil sample coordinates (metres), [Ni]
  // symmetric fold (fold = 1): M, N, K above are the folded sizes; the DFT side's output index a
  // pairs with mirror_n - 1 - a, the contracted index k with K_full - 1 - k (kodd: K_full odd, its
  // middle term has no partner). Output columns c are stored at c < out_h ? c : c + out_s.
  int fold;
  int mirror_n;
  int kodd;
  int out_h, out_s;
  // grouped launches of a multi-problem plan: offset of the problem's star table in the call's
  // packed sources (the launch passes the base; `sources` above is unused there)
  long long src_off;
};

// Tile shape of one GEMM launch: 4 waves (2 x 2), each WM x WN blocks of 16 x 16.
struct TileShape {
  int wm, wn;
  int bm() const { return 32 * wm; }
  int bn() const { return 32 * wn; }
};

// Tile shapes compiled for every stage and precision (the autotuner's candidates).
constexpr TileShape kTileShapes[] = {{4, 4}, {3, 3}, {2, 2}, {4, 2}, {2, 4}, {2, 1}, {1, 2}, {1, 1}, {4, 1}, {1, 4}};

// ---- grouped launches of a multi-problem plan: one launch per stage over every problem
// Entry of a grouped launch's block table: the problem and the block's coordinates in the
// problem's own grid.
struct GroupBlock {
  int k, x, y, z;
};

// Base pointers of one call's packed caller arrays (problem k's arrays start at its element
// offsets, dlx_offsets), and the loss's scalars.
struct GroupCall {
  const float* transmission;
  const float* zbasis;
  const float* coeffs;
  const float* sources;
  const float* flat;
  const float* intrapixel;
  const float* data;
  float* binned;
  float* model;
  float* r;
  double* loss;
  double* grad_flat;
  double* grad_zernike;
  double* grad_sources;
  int kind;
  double mu, inv_s2;
};

// Per-problem arguments of the grouped small kernels (plan-owned pointers, sizes, and the
// offsets of the problem's arrays in the call's packed arrays).
struct PrepArgs {   // OPD, A^2 partial sums, tilt vectors (prep_kernel)
  int Nz, Ni, nb_opd, n_norm, L, ldt;
  long long npix, n_tilt, tplane;
  double* opd;
  double* norm_part;
  const WlInfo* wl;
  const double* x;
  float* tx;
  float* ty;
  long long o_trans, o_z, o_c, o_src;
};
constexpr int kPupilGroupWl = 8;   // wavelengths per block of the grouped pupil launch
struct PupilArgs {   // per-wavelength pupil fields (pupil_kernel)
  const double* opd;
  const float* screen;
  const double* norm_part;
  int n_norm, Ni, ldp, h, L;
  const WlInfo* wl;
  float* P0T;
  long long plane, by_wl, o_trans;
};
struct BinLossArgs {   // binning, model, loss, residual, seed weights of a one-frame problem (bin_loss_kernel)
  const float* E;
  long long plane, by_psf;
  int ld, S, L, Q, Nd, fh, fs, ldg, nb;
  const WlInfo* wl;
  long long kst, g_by_frame;
  float* bs;
  double* blk;
  int* status;
  float* G;
  double* flux;
  long long o_src, o_flat, o_k, o_img;
};
struct GradArgs {   // dL/dOPD, its Zernike projection and the final sums (gopd, zproj, finalize)
  const float* gpart;
  int G;
  long long npix;
  double* gopd;
  int Nz, nchunks;
  long long zchunk;
  double* zpart;
  const double* flux;
  int flux_blocks, tiles_b4, L, FS, nloss;
  const double* pos;
  const double* lossblk;
  long long o_z, o_c, o_src, o_loss;
};

hipError_t launch_prep_group(const PrepArgs* args, const GroupBlock* tab, int n_blocks, const GroupCall& call,
                             hipStream_t st);
hipError_t launch_pupil_group(const PupilArgs* args, const GroupBlock* tab, int n_blocks, const GroupCall& call,
                              hipStream_t st);
// qt: the compiled oversampling of the bin_loss_kernel instance (1, 2, 4, or 0 = any)
hipError_t launch_bin_loss_group(int qt, const BinLossArgs* args, const GroupBlock* tab, int n_blocks,
                                 const GroupCall& call, hipStream_t st);
hipError_t launch_grad_group(const GradArgs* args, const GroupBlock* gopd_tab, int n_gopd, const GroupBlock* z_tab,
                             int n_z, const GroupBlock* fin_tab, int n_fin, const GroupCall& call, hipStream_t st);

int loss_block_count(long long npix);
hipError_t launch_loss_plain(int nf, long long npix, const float* model, const float* binned, const float* data,
                             const float* flat, int kind, double mu, double sigma, float* r, double* gflat,
                             double* blk, int* status, double* loss, hipStream_t st);
hipError_t launch_gemm(int kind, int prec, TileShape ts, const GemmArgs& a, int n_wg, hipStream_t st);
// One folded stage over many problems: n_wg workgroups, tab[g] = (problem, its logical workgroup),
// args = per-problem arguments in device memory, sources = the call's packed star table.
hipError_t launch_gemm_group(int kind, int prec, TileShape ts, const GemmArgs* args, const int2* tab, int n_wg,
                             const float* sources, hipStream_t st);
bool tile_supported(int kind, int prec, bool fold, TileShape ts);

struct GroupPlan;

}  // namespace dlx

struct dlx_plan {
  // several independent problems: one sub-plan each, run on side streams
  std::vector<dlx_plan*> subs;
  std::vector<dlx_offsets> offs;
  std::vector<hipStream_t> side;
  std::vector<int> order, lane;   // issue order (largest first) and side stream of each problem
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  bool multi() const { return !subs.empty(); }
  // grouped launches (one per stage over every problem) when every problem qualifies; null otherwise
  dlx::GroupPlan* group = nullptr;
  // problem. In integer-dither mode the MFT stages see one frame of an enlarged
  // detector (F = 1, Nd = N_det + 2 margin, No = Q Nd) and the images are
  // F_img windows of N_det_img pixels; otherwise F_img = F and Nd_img = Nd.
  int Ni, No, Q, Nd, L, S, F, Nz, Nmap;
  int F_img = 0, Nd_img = 0;
  bool dither = false;
  int margin = 0;
  std::vector<int> win;   // [F_img][2] window corners (row, col) in the enlarged plane
  double D, du, dx;
  std::vector<double> lam, wts;
  dlx_precision prec;
  int bf16() const { return prec == DLX_BF16X3 ? 1 : 0; }
  // padded leading dimensions
  int ldNi, ldNo;
  // symmetric fold of the MFT products (off: dense complex products). Folded data rows keep
  // columns c < h at c and move c >= h to c + ld - N, with h = ceil(N / 2).
  bool fold = true;
  int hNi() const { return (Ni + 1) / 2; }
  int hNo() const { return (No + 1) / 2; }
  int sNi() const { return fold ? ldNi - Ni : 0; }
  int sNo() const { return fold ? ldNo - No : 0; }
  // chunking
  int frames_per_chunk;
  int n_chunks;
  int chunk_psf;        // PSFs in a full chunk
  int n_psf;
  // tiles
  dlx::TileShape ts_f1, ts_f2, ts_b3, ts_b4;
  int b4_gsize, b4_groups_max, b4_ksplit = 1;
  int b4_gsize_default = 1, b4_groups_alloc = 1;   // B4: the heuristic group size; groups d_gpart holds
  int b4_ksplit_tuned = 0;   // B4's K split chosen by the autotuner (0: the heuristic)
  // device memory
  void* pool = nullptr;
  size_t pool_bytes = 0;
  dlx::WlInfo* d_wl = nullptr;
  float* d_MN = nullptr;   // [L][No][ldNi] planar
  float* d_MT = nullptr;   // [L][Ni][ldNo] planar
  double* d_x = nullptr;   // [Ni]
  double* d_opd = nullptr;    // OPD [Ni*Ni]
  float* d_screen = nullptr;  // static pupil phase screen, radians [Ni*Ni] (zero unless set)
  float* d_maptmp = nullptr;  // [Nmap][Ni]
  double* d_norm = nullptr;   // partial sums of A^2 [n_norm_part]
  int n_norm_part = 1;
  float* d_P0T = nullptr;  // [L][Ni][ldNi] planar
  float* d_tx = nullptr;   // [n_psf][ldNi] planar
  float* d_ty = nullptr;
  float* d_T = nullptr;    // [chunk_psf][No][ldNi] planar
  float* d_Y = nullptr;    // [chunk_psf][No][ldNo] planar FP32: the focal fields E
  float* d_UT = nullptr;   // [chunk_psf][Ni][ldNo] planar
  float* d_G = nullptr;    // seed weights G = K flat r [frames_per_chunk][No][ldNo]
  float* d_bs = nullptr;   // per-source binned sum_l w_l K|E|^2 [frames_per_chunk][S][Nd*Nd]
  float* d_Bbig = nullptr; // integer-dither mode: binned enlarged plane [Nd*Nd]
  int* d_win = nullptr;    // integer-dither mode: window corners [F_img][2]
  float* d_gpart = nullptr;    // [b4_groups_max * b4_ksplit][Ni*Ni], room for b4_groups_alloc groups
  double* d_gopd = nullptr;    // [Ni*Ni]
  double* d_flux = nullptr;    // flux gradient partials [F][S][seed blocks]
  double* d_kpart = nullptr;   // intra-pixel kernel gradient partials [F][seed blocks][Q*Q]
  double* d_pos = nullptr;     // [n_psf][b4_ksplit][tiles_b4][2]
  double* d_lossblk = nullptr; // [loss blocks]
  double* d_tmp2 = nullptr;    // [Ni][Nmap] for the map gradient
  double* d_zpart = nullptr;   // Zernike projection partials [chunks][Nz]
  int* d_status = nullptr;
  int loss_blocks = 0;
  int seed_blocks = 0;   // pixel blocks of the seed-weight kernel
  // partial counts of the last launches that wrote them (flux partials per (frame, star); loss
  // partials per chunk): seed kernels and loss_kernel use 256-pixel blocks, bin_loss_kernel 64
  int flux_blocks = 0, lossblk_chunk = 0;
  bool seed_pass = false; // form Y = w phi G E in a separate pass (dense plans with large frames, or on request) instead of in B3's loader
  // stage timing (diagnostics)
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  int ev_used = 0;
  struct Rec { int stage; int e0, e1; long long psfs; };
  std::vector<Rec> recs;
  double stage_ms[DLX_N_STAGES] = {};
  long long stage_launches[DLX_N_STAGES] = {};
  long long stage_psfs[DLX_N_STAGES] = {};
  int tiles_b4 = 0;
  int tiles_b4_cap = 0, ksplit_cap = 1;   // sizes the partial-sum buffers
  float* d_tune = nullptr;
  bool tuned = false;
  bool k_per_pixel = false;   // one intra-pixel kernel per detector pixel ([Nd][Nd][Q][Q])
  bool store_fields = false;  // keep E and the per-star binned images from forward to backward
  bool fields_valid = false;  // the workspace holds the fields of the last dlx_psf_forward
  // captured evaluation
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
};
