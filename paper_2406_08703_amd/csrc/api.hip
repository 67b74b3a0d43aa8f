// C ABI of libdlx (include/dlx.h): validation, plan construction (tiles,
// chunking, workspace, DFT matrices) and the forward / loss / backward
// launch sequences. All device work is enqueued on the caller's stream.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>

#include "dlx_internal.h"

namespace dlx {
hipError_t launch_dft(dlx_plan* p, hipStream_t st);
hipError_t launch_zero(float* x, long long n, hipStream_t st);
hipError_t launch_prep(dlx_plan* p, const float* A, const float* Z, const float* Bm, const float* c, const float* C,
                       const float* sources, hipStream_t st);
hipError_t launch_intensity(dlx_plan* p, int f0, int nf, const float* sources, const float* intrapixel,
                            const float* flat, float* binned, float* model, hipStream_t st);
hipError_t launch_seed(dlx_plan* p, int f0, int nf, const float* flat, const float* resid, const float* intrapixel,
                       hipStream_t st);
hipError_t launch_seed_apply(dlx_plan* p, int f0, int nf, const float* sources, hipStream_t st);
hipError_t launch_window(dlx_plan* p, const float* flat, float* binned, float* model, hipStream_t st);
hipError_t launch_seed_gather(dlx_plan* p, const float* flat, const float* resid, const float* intrapixel,
                              hipStream_t st);
hipError_t launch_loss(dlx_plan* p, int f0, int nf, int chunk, const float* model, const float* binned,
                       const float* data, const float* flat, int kind, double mu, double sigma, float* r, double* gflat,
                       const float* const* seed_intrapixel_or_none, hipStream_t st);
hipError_t launch_loss_final(dlx_plan* p, int n_chunks, double* loss, hipStream_t st);
hipError_t launch_bin_loss(dlx_plan* p, int f0, int nf, int chunk, const float* sources, const float* intrapixel,
                           const float* flat, const float* data, int kind, double mu, double sigma, float* binned,
                           float* model, float* r, double* gflat, hipStream_t st);
hipError_t launch_grad_reduce(dlx_plan* p, const float* Z, const float* Bm, double* gz, double* gmap, double* gsrc,
                              double* loss, int loss_chunks, double* gK, hipStream_t st);
hipError_t launch_kgrad(dlx_plan* p, int f0, int nf, const float* sources, const float* flat, const float* resid,
                        double* gK, hipStream_t st);
int loss_block_count(long long npix);
int seed_block_count(long long npix);
int zproj_chunks(long long npix, int Nz);
int bin_loss_block_count(long long npix);
}  // namespace dlx

using namespace dlx;

namespace {

constexpr size_t kDefaultChunkBudget = size_t(8) << 30;  // bytes of per-chunk intermediates
constexpr int kTargetWG = 1024;
constexpr int kMaxKgradQ = 4;   // the intra-pixel gradient kernel is compiled for Q <= 4
// A frame's seed weights larger than this (bytes) are applied in a separate
// pass rather than streamed by every B3 workgroup (about one XCD's L2).
constexpr size_t kSeedFuseMaxBytes = size_t(4) << 20;

#define DLX_HIP(expr)                        \
  do {                                       \
    if ((expr) != hipSuccess) return DLX_ERR_HIP; \
  } while (0)

int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Pick the output tile of a stage. A wave owns (16 w) x (16 w) outputs and
// the workgroup (32 w) x (32 w); w = 4 (128 x 128) is used when it still
// gives enough workgroups to fill the chip, otherwise the smallest valid w.
// With q > 1 the wave tile edge must be divisible by q, so that each
// detector pixel's q x q focal samples stay inside one wave's tile.
TileShape choose_tile(int M, int N, long long items, int q, bool fold = false) {
  const int cand[3] = {4, 3, 2};
  int smallest = 0;
  for (int w : cand) {
    if (q > 1 ? ((16 * w) % q != 0) : (w == 3)) continue;
    if (fold && w == 4) continue;   // folded 128 x 128 tiles are not compiled
    const long long wg = (long long)ceil_div(M, 32 * w) * ceil_div(N, 32 * w) * items;
    if (wg >= 2 * kTargetWG) return TileShape{w, w};
    smallest = w;
  }
  return TileShape{smallest, smallest};
}

struct Pool {
  char* base;
  size_t off;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += sizeof(T) * count;
    return p;
  }
};

void layout(dlx_plan* p, Pool& pool) {
  const size_t L = p->L, Ni = p->Ni, No = p->No, ldNi = p->ldNi, ldNo = p->ldNo, CP = p->chunk_psf;
  p->d_wl = pool.take<WlInfo>(L);
  p->d_MN = pool.take<float>(2 * L * No * ldNi);
  p->d_MT = pool.take<float>(2 * L * Ni * ldNo);
  p->d_x = pool.take<double>(Ni);
  p->d_opd = pool.take<double>((size_t)Ni * Ni);
  p->d_screen = pool.take<float>((size_t)Ni * Ni);
  p->d_maptmp = pool.take<float>(std::max<size_t>(1, (size_t)p->Nmap * Ni));
  p->d_norm = pool.take<double>(p->n_norm_part);
  p->d_P0T = pool.take<float>(2 * L * Ni * ldNi);
  p->d_tx = pool.take<float>(2 * (size_t)p->n_psf * ldNi);
  p->d_ty = pool.take<float>(2 * (size_t)p->n_psf * ldNi);
  p->d_T = pool.take<float>(2 * CP * No * ldNi);
  p->d_Y = pool.take<float>(2 * CP * No * ldNo);
  p->d_UT = pool.take<float>(2 * CP * Ni * ldNo);
  p->d_G = pool.take<float>((size_t)p->frames_per_chunk * No * ldNo);
  p->d_bs = pool.take<float>((size_t)p->frames_per_chunk * p->S * p->Nd * p->Nd);
  if (p->dither) {
    p->d_Bbig = pool.take<float>((size_t)p->Nd * p->Nd);
    p->d_win = pool.take<int>(p->win.size());
  }
  p->d_gpart = pool.take<float>((size_t)p->b4_groups_alloc * p->ksplit_cap * Ni * Ni);
  p->d_gopd = pool.take<double>(Ni * Ni);
  const size_t pix64 = ((size_t)p->Nd * p->Nd + 63) / 64;   // bin_loss_kernel's pixel blocks
  p->d_flux = pool.take<double>((size_t)p->F * p->S * std::max<size_t>(p->seed_blocks, pix64));
  p->d_kpart = pool.take<double>((size_t)p->F * p->seed_blocks * p->Q * p->Q);
  p->d_pos = pool.take<double>((size_t)p->n_psf * p->ksplit_cap * p->tiles_b4_cap * 2);
  p->d_lossblk = pool.take<double>(std::max<size_t>(p->loss_blocks, pix64) * p->n_chunks);
  p->d_tmp2 = pool.take<double>(std::max<size_t>(1, Ni * (size_t)p->Nmap));
  p->d_zpart = pool.take<double>((size_t)std::max(1, zproj_chunks((long long)Ni * Ni, p->Nz)) * std::max(1, p->Nz));
  p->d_status = pool.take<int>(1);
  // autotuning stand-in for the caller's sources, read by B3 [F][S][3]
  p->d_tune = pool.take<float>((size_t)p->F * p->S * 3);
}

// T, E and U^T of one PSF
size_t per_psf_bytes(const dlx_plan* p) {
  return sizeof(float) * 2 * ((size_t)p->No * p->ldNi + (size_t)p->No * p->ldNo + (size_t)p->Ni * p->ldNo);
}

// seed weights and per-source binned images of one frame
size_t per_frame_bytes(const dlx_plan* p) {
  return sizeof(float) * ((size_t)p->No * p->ldNo + (size_t)p->S * p->Nd * p->Nd);
}

bool ok_ptr(const void* q) { return q != nullptr; }

GemmArgs base_args(const dlx_plan* p, int f0, int nframes) {
  GemmArgs a;
  std::memset(&a, 0, sizeof(a));
  a.L = p->L;
  a.S = p->S;
  a.psf0 = f0 * p->S * p->L;
  a.frame0 = f0;
  a.n_chunk_psf = nframes * p->S * p->L;
  a.tx = p->d_tx;
  a.ty = p->d_ty;
  a.tilt_plane = (long long)p->n_psf * p->ldNi;
  a.ldt = p->ldNi;
  a.p0t = p->d_P0T;
  a.p0_plane = (long long)p->Ni * p->ldNi;
  a.p0_by_wl = 2LL * p->Ni * p->ldNi;
  a.ldp = p->ldNi;
  a.wl = p->d_wl;
  a.xcoord = p->d_x;
  return a;
}

Operand op_MN(const dlx_plan* p) {
  return Operand{p->d_MN, (long long)p->L * p->No * p->ldNi, (long long)p->No * p->ldNi, 0, p->ldNi};
}
Operand op_MT(const dlx_plan* p) {
  return Operand{p->d_MT, (long long)p->L * p->Ni * p->ldNo, (long long)p->Ni * p->ldNo, 0, p->ldNo};
}
Operand op_T(const dlx_plan* p) {
  return Operand{p->d_T, (long long)p->chunk_psf * p->No * p->ldNi, 0, (long long)p->No * p->ldNi, p->ldNi};
}
// the stored focal fields E (FP32 in both arithmetics)
Operand op_E(const dlx_plan* p) {
  return Operand{p->d_Y, (long long)p->chunk_psf * p->No * p->ldNo, 0, (long long)p->No * p->ldNo, p->ldNo};
}
Operand op_UT(const dlx_plan* p) {
  return Operand{p->d_UT, (long long)p->chunk_psf * p->Ni * p->ldNo, 0, (long long)p->Ni * p->ldNo, p->ldNo};
}

int wg_count(const GemmArgs& a) { return a.tiles_m * a.tiles_n * a.n_items; }

// ---- stage timing (diagnostics): event pairs bracket each stage on the call's stream
constexpr int kEventPool = 512;

hipError_t flush_records(dlx_plan* p) {
  for (const auto& r : p->recs) {
    hipError_t e = hipEventSynchronize(p->ev_pool[r.e1]);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, p->ev_pool[r.e0], p->ev_pool[r.e1]);
    if (e != hipSuccess) return e;
    p->stage_ms[r.stage] += ms;
    p->stage_launches[r.stage] += 1;
    p->stage_psfs[r.stage] += r.psfs;
  }
  p->recs.clear();
  p->ev_used = 0;
  return hipSuccess;
}

struct Stage {
  dlx_plan* p;
  hipStream_t st;
  int stage;
  long long psfs;
  int e0 = -1;
  Stage(dlx_plan* p_, hipStream_t st_, int stage_, long long psfs_) : p(p_), st(st_), stage(stage_), psfs(psfs_) {
    if (!p->profiling) return;
    if (p->ev_used + 2 > (int)p->ev_pool.size() && flush_records(p) != hipSuccess) return;
    e0 = p->ev_used;
    p->ev_used += 2;
    if (hipEventRecord(p->ev_pool[e0], st) != hipSuccess) e0 = -1;
  }
  ~Stage() {
    if (e0 < 0) return;
    if (hipEventRecord(p->ev_pool[e0 + 1], st) == hipSuccess) p->recs.push_back({stage, e0, e0 + 1, psfs});
  }
};

void set_tiles(GemmArgs& a, TileShape ts) {
  a.tiles_m = ceil_div(a.M, ts.bm());
  a.tiles_n = ceil_div(a.N, ts.bn());
}

// Symmetric fold of one stage: the DFT side's output rows and the contracted length are halved
// (mirror_n and the contracted length k_full are the unfolded sizes); output columns c >= out_h
// are stored at c + out_s.
void set_fold(const dlx_plan* p, GemmArgs& a, int mirror_n, int k_full, int out_h, int out_s) {
  if (!p->fold) return;
  a.fold = 1;
  a.mirror_n = mirror_n;
  a.kodd = k_full & 1;
  a.out_h = out_h;
  a.out_s = out_s;
}

// F1: T = M_l P for every PSF of frames [f0, f0 + nf)
GemmArgs args_f1(dlx_plan* p, int f0, int nf) {
  GemmArgs a = base_args(p, f0, nf);
  a.M = p->fold ? p->hNo() : p->No;
  a.N = p->Ni;
  a.K = p->fold ? p->hNi() : p->Ni;
  set_fold(p, a, p->No, p->Ni, p->hNi(), p->sNi());
  a.n_items = a.n_chunk_psf;
  a.A = op_MN(p);
  a.B = Operand{p->d_P0T, (long long)p->Ni * p->ldNi, 2LL * p->Ni * p->ldNi, 0, p->ldNi};
  a.out = p->d_T;
  a.out_plane = op_T(p).plane;
  a.out_by_psf = op_T(p).by_psf;
  a.ldo = p->ldNi;
  set_tiles(a, p->ts_f1);
  return a;
}

hipError_t run_f1(dlx_plan* p, int f0, int nf, hipStream_t st) {
  const GemmArgs a = args_f1(p, f0, nf);
  return launch_gemm(KIND_F1, p->bf16(), p->ts_f1, a, wg_count(a), st);
}

GemmArgs e_args(dlx_plan* p, int f0, int nf, TileShape ts);

// F2 over frames [f0, f0 + nf): E = c T M^T into the Y buffer.
GemmArgs args_f2(dlx_plan* p, int f0, int nf) {
  GemmArgs a = e_args(p, f0, nf, p->ts_f2);
  a.n_items = nf * p->S * p->L;
  if (p->fold) {
    a.N = p->hNo();
    a.K = p->hNi();
    set_fold(p, a, p->No, p->Ni, p->hNo(), p->sNo());
    set_tiles(a, p->ts_f2);
  }
  a.out = p->d_Y;
  a.out_plane = (long long)p->chunk_psf * p->No * p->ldNo;
  a.out_by_psf = (long long)p->No * p->ldNo;
  a.ldo = p->ldNo;
  return a;
}

hipError_t run_f2(dlx_plan* p, int f0, int nf, hipStream_t st) {
  const GemmArgs a = args_f2(p, f0, nf);
  return launch_gemm(KIND_F2, p->bf16(), p->ts_f2, a, wg_count(a), st);
}

// B3 over frames [f0, f0 + nf): U^T = conj(M)^T Y^T with the seed Y = w phi G E
// formed in the loader from E and the seed weights G.
GemmArgs args_b3(dlx_plan* p, int f0, int nf, const float* sources) {
  GemmArgs a = base_args(p, f0, nf);
  a.M = p->fold ? p->hNi() : p->Ni;
  a.N = p->No;
  a.K = p->fold ? p->hNo() : p->No;
  set_fold(p, a, p->Ni, p->No, p->hNo(), p->sNo());
  a.n_items = nf * p->S * p->L;
  a.A = op_MT(p);
  a.conj_a = 1;
  a.B = op_E(p);
  a.sources = sources;
  a.seedw = p->seed_pass ? nullptr : p->d_G;
  a.seedw_by_frame = (long long)p->No * p->ldNo;
  a.out = p->d_UT;
  a.out_plane = op_UT(p).plane;
  a.out_by_psf = op_UT(p).by_psf;
  a.ldo = p->ldNo;
  set_tiles(a, p->ts_b3);
  return a;
}

hipError_t run_b3(dlx_plan* p, int f0, int nf, const float* sources, hipStream_t st) {
  const GemmArgs a = args_b3(p, f0, nf, sources);
  return launch_gemm(KIND_B3, p->bf16(), p->ts_b3, a, wg_count(a), st);
}

// B4 over frames [f0, f0 + nf) of chunk c: W = c M^H U, phase gradient and position sums.
GemmArgs args_b4(dlx_plan* p, int c, int f0, int nf) {
  const int nc = nf * p->S * p->L;
  GemmArgs a = base_args(p, f0, nf);
  a.M = p->fold ? p->hNi() : p->Ni;
  a.N = p->Ni;
  a.K = p->fold ? p->hNo() : p->No;
  set_fold(p, a, p->Ni, p->No, p->Ni, 0);
  a.A = op_MT(p);
  a.conj_a = 1;
  a.B = op_UT(p);
  a.group_size = p->b4_gsize;
  a.ksplit = p->b4_ksplit;
  a.groups = ceil_div(nc, p->b4_gsize);
  a.n_items = a.groups * p->b4_ksplit;
  a.part = p->d_gpart;
  a.accumulate = c > 0;
  a.red = p->d_pos;
  set_tiles(a, p->ts_b4);
  return a;
}

hipError_t run_b4(dlx_plan* p, int c, int f0, int nf, hipStream_t st) {
  const GemmArgs a = args_b4(p, c, f0, nf);
  return launch_gemm(KIND_B4, p->bf16(), p->ts_b4, a, wg_count(a), st);
}

// B3 and B4 of chunk c.
hipError_t run_adjoint(dlx_plan* p, int c, int f0, int nf, const float* sources, hipStream_t st) {
  const int nc = nf * p->S * p->L;
  {
    Stage sg(p, st, DLX_STAGE_B3, nc);
    hipError_t e = run_b3(p, f0, nf, sources, st);
    if (e != hipSuccess) return e;
  }
  Stage sg(p, st, DLX_STAGE_B4, nc);
  return run_b4(p, c, f0, nf, st);
}

// Tile-dependent derived sizes: partial-sum tile counts and B4's split of K (`ksplit` > 0 sets it,
// as the autotuner does; otherwise K = No is split when the groups alone cannot fill the chip,
// keeping >= 128 per split).
void derive_tiles(dlx_plan* p, int ksplit = 0) {
  p->tiles_b4 = ceil_div(p->fold ? p->hNi() : p->Ni, p->ts_b4.bm()) * ceil_div(p->Ni, p->ts_b4.bn());
  if (ksplit > 0) {
    p->b4_ksplit = ksplit;
    return;
  }
  const long long wg = (long long)p->tiles_b4 * p->b4_groups_max;
  int ks = 1;
  const int kb4 = p->fold ? p->hNo() : p->No;
  while (ks < 4 && wg * ks < kTargetWG && kb4 / (2 * ks) >= 128) ks *= 2;
  p->b4_ksplit = ks;
}

// ---- autotuner: time every compiled tile shape per MFT stage on chunk 0
hipError_t run_stage_for_tuning(dlx_plan* p, int kind, hipStream_t st) {
  const int nf = std::min(p->frames_per_chunk, p->F);
  switch (kind) {
    case KIND_F1: return run_f1(p, 0, nf, st);
    case KIND_F2: return run_f2(p, 0, nf, st);
    case KIND_B3: return run_b3(p, 0, nf, p->d_tune, st);
    default: return run_b4(p, 0, 0, nf, st);
  }
}

TileShape* stage_tile(dlx_plan* p, int kind) {
  switch (kind) {
    case KIND_F1: return &p->ts_f1;
    case KIND_F2: return &p->ts_f2;
    case KIND_B3: return &p->ts_b3;
    default: return &p->ts_b4;
  }
}

// Runs on the zeroed workspace with the DFT matrices built, so every operand is finite.
hipError_t autotune(dlx_plan* p) {
  hipError_t e;
  hipEvent_t t0, t1;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&t1)) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return e;
  }
  const int kinds[4] = {KIND_F1, KIND_F2, KIND_B3, KIND_B4};
  const char* env = std::getenv("DLX_TUNE_LOG");   // diagnostics: print every candidate's time
  const bool log = env && env[0] == '1';
  for (int kind : kinds) {
    TileShape* ts = stage_tile(p, kind);
    TileShape best = *ts;
    int best_ks = 0, best_gs = p->b4_gsize;
    float best_ms = 1e30f;
    // B4 also tries each split of its K (= No) into 1, 2 or 4 ranges of at least 64, and groups of
    // the heuristic size, twice and four times it
    const int n_ks = kind == KIND_B4 ? 3 : 1, n_gs = kind == KIND_B4 ? 3 : 1;
    const int n_cand = (int)(sizeof(kTileShapes) / sizeof(kTileShapes[0])) * n_ks * n_gs;
    for (int ci = 0; ci < n_cand && e == hipSuccess; ++ci) {
      const TileShape& cand = kTileShapes[ci / (n_ks * n_gs)];
      const int ks = kind == KIND_B4 ? (1 << (ci / n_gs % n_ks)) : 0;
      if (ks > 1 && (p->fold ? p->hNo() : p->No) / ks < 64) continue;
      if (!tile_supported(kind, p->bf16(), p->fold, cand)) continue;
      if (kind == KIND_B4) {
        const int gs = std::min(p->chunk_psf, p->b4_gsize_default << (ci % n_gs));
        if (ci % n_gs > 0 && gs == std::min(p->chunk_psf, p->b4_gsize_default << (ci % n_gs - 1))) continue;
        p->b4_gsize = gs;
        p->b4_groups_max = ceil_div(p->chunk_psf, gs);
      }
      *ts = cand;
      derive_tiles(p, ks);
      if ((e = run_stage_for_tuning(p, kind, nullptr)) != hipSuccess) break;   // warm-up
      if ((e = hipEventRecord(t0, nullptr)) != hipSuccess) break;
      for (int r = 0; r < 2 && e == hipSuccess; ++r) e = run_stage_for_tuning(p, kind, nullptr);
      if (e != hipSuccess) break;
      if ((e = hipEventRecord(t1, nullptr)) != hipSuccess) break;
      if ((e = hipEventSynchronize(t1)) != hipSuccess) break;
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
      if (log)
        std::fprintf(stderr, "dlx tune: stage %d tile %dx%d ksplit %d group %d: %.4f ms per launch\n", kind,
                     cand.bm(), cand.bn(), p->b4_ksplit, p->b4_gsize, ms / 2);
      if (ms < best_ms) {
        best_ms = ms;
        best = cand;
        best_ks = ks;
        best_gs = p->b4_gsize;
      }
    }
    *ts = best;
    if (kind == KIND_B4) {
      p->b4_gsize = best_gs;
      p->b4_groups_max = ceil_div(p->chunk_psf, best_gs);
    }
    derive_tiles(p, best_ks);
    if (kind == KIND_B4) p->b4_ksplit_tuned = best_ks;
    if (e != hipSuccess) break;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  p->tuned = e == hipSuccess;
  return e;
}

// Tuned tiles per problem shape and device, shared by every plan of the
// process, so plans of a shape already seen skip the timing runs. With the
// environment variable DLX_TUNE_CACHE naming a file, that file is the cache
// instead: tuned shapes are looked up in it and appended to it, one line each,
// so the choice carries across processes (lines whose tiles are not compiled
// for their stage, or that do not parse, are ignored).
using TuneKey = std::array<long long, 12>;
std::mutex g_tune_mu;
struct Tuned {
  std::array<TileShape, 4> tiles;   // F1, F2, B3, B4
  int b4_ksplit;
  int b4_gsize;                     // PSFs per B4 group
};
std::map<TuneKey, Tuned> g_tune;

TuneKey tune_key(const dlx_plan* p) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return {dev, (long long)p->prec, p->Ni, p->No, p->Q, p->L, p->S, p->F, p->frames_per_chunk, p->Nz, p->Nmap,
          (p->seed_pass ? 1 : 0) | (p->fold ? 2 : 0)};
}

// "dlx-tune-v2 <arch> <CUs> <prec Ni No Q L S F frames_per_chunk Nz Nmap flags>" of the cache file:
// the device is named by its architecture and compute-unit count, not by its index.
bool disk_key(const dlx_plan* p, char* buf, size_t n) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  char arch[64];
  int k = 0;
  for (const char* c = prop.gcnArchName; *c && *c != ':' && k < 63; ++c) arch[k++] = *c;
  arch[k] = 0;
  const TuneKey t = tune_key(p);
  const int w = std::snprintf(buf, n, "dlx-tune-v2 %s %d %lld %lld %lld %lld %lld %lld %lld %lld %lld %lld %lld",
                              arch, prop.multiProcessorCount, t[1], t[2], t[3], t[4], t[5], t[6], t[7], t[8], t[9],
                              t[10], t[11]);
  return w > 0 && (size_t)w < n;
}

bool tuned_valid(const dlx_plan* p, const Tuned& t) {
  const int kinds[4] = {KIND_F1, KIND_F2, KIND_B3, KIND_B4};
  for (int i = 0; i < 4; ++i)
    if (!tile_supported(kinds[i], p->bf16(), p->fold, t.tiles[i])) return false;
  if (t.b4_gsize < 1 || ceil_div(p->chunk_psf, t.b4_gsize) > p->b4_groups_alloc) return false;
  return t.b4_ksplit == 0 || t.b4_ksplit == 1 || t.b4_ksplit == 2 || t.b4_ksplit == 4;
}

bool disk_lookup(const dlx_plan* p, const char* path, Tuned* out) {
  char key[256];
  if (!disk_key(p, key, sizeof key)) return false;
  std::FILE* f = std::fopen(path, "r");
  if (!f) return false;
  const size_t kl = std::strlen(key);
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {   // the last valid line for the key wins
    if (std::strncmp(line, key, kl) != 0 || std::strncmp(line + kl, " : ", 3) != 0) continue;
    int v[10];
    if (std::sscanf(line + kl + 3, "%d %d %d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5],
                    &v[6], &v[7], &v[8], &v[9]) != 10)
      continue;
    Tuned t{{TileShape{v[0], v[1]}, TileShape{v[2], v[3]}, TileShape{v[4], v[5]}, TileShape{v[6], v[7]}}, v[8], v[9]};
    if (!tuned_valid(p, t)) continue;
    *out = t;
    found = true;
  }
  std::fclose(f);
  return found;
}

void disk_store(const dlx_plan* p, const char* path, const Tuned& t) {
  char key[256];
  if (!disk_key(p, key, sizeof key)) return;
  std::FILE* f = std::fopen(path, "a");
  if (!f) return;   // an unwritable cache only costs the next process its tuning
  std::fprintf(f, "%s : %d %d %d %d %d %d %d %d %d %d\n", key, t.tiles[0].wm, t.tiles[0].wn, t.tiles[1].wm,
               t.tiles[1].wn, t.tiles[2].wm, t.tiles[2].wn, t.tiles[3].wm, t.tiles[3].wn, t.b4_ksplit, t.b4_gsize);
  std::fclose(f);
}

void apply_tuned(dlx_plan* p, const Tuned& t) {
  p->ts_f1 = t.tiles[0];
  p->ts_f2 = t.tiles[1];
  p->ts_b3 = t.tiles[2];
  p->ts_b4 = t.tiles[3];
  p->b4_ksplit_tuned = t.b4_ksplit;
  p->b4_gsize = t.b4_gsize;
  p->b4_groups_max = ceil_div(p->chunk_psf, t.b4_gsize);
  derive_tiles(p, p->b4_ksplit_tuned);
  p->tuned = true;
}

hipError_t autotune_cached(dlx_plan* p) {
  const char* path = std::getenv("DLX_TUNE_CACHE");
  const bool disk = path && path[0];
  const TuneKey key = tune_key(p);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    Tuned t;
    if (disk) {
      if (disk_lookup(p, path, &t)) {
        apply_tuned(p, t);
        return hipSuccess;
      }
    } else {
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        apply_tuned(p, it->second);
        return hipSuccess;
      }
    }
  }
  const hipError_t e = autotune(p);
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const Tuned t{{p->ts_f1, p->ts_f2, p->ts_b3, p->ts_b4}, p->b4_ksplit_tuned, p->b4_gsize};
    if (disk)
      disk_store(p, path, t);
    else
      g_tune[key] = t;
  }
  return e;
}

GemmArgs e_args(dlx_plan* p, int f0, int nf, TileShape ts) {
  GemmArgs a = base_args(p, f0, nf);
  a.M = p->No;
  a.N = p->No;
  a.K = p->Ni;
  a.A = op_T(p);
  a.B = op_MN(p);
  set_tiles(a, ts);
  return a;
}

}  // namespace

extern "C" dlx_status dlx_plan_destroy(dlx_plan* p);
extern "C" dlx_status dlx_plan_create(const dlx_problem_desc* probs, int32_t n_probs, dlx_precision precision,
                                      int32_t flags, size_t workspace_limit_bytes, dlx_plan** out);

namespace {

// ---- grouped launches: every stage of dlx_eval as one launch over all problems of the plan.
// Used when every problem has one frame, no bicubic map and no integer dithers, and the plan folds
// its products with the seed formed in B3's loader (no flags beyond NO_AUTOTUNE). Per-problem
// arguments and block tables sit in device memory, built at plan creation; each call passes only
// the base pointers of its packed arrays, so a captured graph replays with the call's pointers.
}  // namespace

namespace dlx {
struct GroupPlan {
  void* dmem = nullptr;         // GEMM arguments, block tables and the tuning star table
  void* dmem_small = nullptr;   // the small stages' arguments and block tables
  TileShape ts[4];     // F1, F2, B3, B4, shared by every problem
  int b4_ks = 1;       // B4's split of K (each problem keeps at least 64 per range)
  int b4_psfs = 32;    // PSFs per B4 group: one launch fills the chip with every problem's tiles, so
                       // a problem needs few groups, and few dL/dOPD partial planes to write and reduce
  std::vector<int> b4_groups_cap;   // each problem's group count its partial-plane buffer holds
  GemmArgs* d_gargs[4] = {};
  int2* d_gtab[4] = {};
  int n_wg[4] = {}, cap_wg[4] = {};
  PrepArgs* d_prep = nullptr;
  GroupBlock* d_prep_tab = nullptr;
  int n_prep = 0;
  PupilArgs* d_pupil = nullptr;
  GroupBlock* d_pupil_tab = nullptr;
  int n_pupil = 0;
  BinLossArgs* d_bl = nullptr;
  GroupBlock* d_bl_tab[5] = {};   // problems by the compiled oversampling of their binning: 1, 2, 3, 4, other
  int n_bl[5] = {}, qt_of[5] = {1, 2, 3, 4, 0};
  GradArgs* d_grad = nullptr;
  GroupBlock *d_gopd_tab = nullptr, *d_z_tab = nullptr, *d_fin_tab = nullptr;
  int n_gopd = 0, n_z = 0, n_fin = 0;
  float* d_tune_src = nullptr;
};
}  // namespace dlx

namespace {

constexpr int kGroupKinds[4] = {KIND_F1, KIND_F2, KIND_B3, KIND_B4};

bool group_eligible(const dlx_problem_desc* probs, int n, int32_t flags) {
  if (!(flags & DLX_FLAG_GROUPED)) return false;
  if (flags & (DLX_FLAG_SEED_PASS | DLX_FLAG_STORE_FIELDS | DLX_FLAG_PIXEL_KERNEL | DLX_FLAG_DENSE_MFT)) return false;
  for (int k = 0; k < n; ++k)
    if (probs[k].frame_dithers || probs[k].n_frames != 1 || probs[k].n_map != 0) return false;
  return true;
}

int b4_split_for(const dlx_plan* q, int ks) {
  while (ks > 1 && q->hNo() / ks < 64) ks /= 2;
  return ks;
}

int bin_class(int Q) { return Q >= 1 && Q <= 4 ? Q - 1 : 4; }

// Stage s's tiles on every sub-plan (B4 with its split), as the grouped launch and the per-problem
// calls of the plan use them.
void group_apply_tiles(dlx_plan* p, int s) {
  GroupPlan& g = *p->group;
  for (size_t k = 0; k < p->subs.size(); ++k) {
    dlx_plan* q = p->subs[k];
    TileShape* t = s == 0 ? &q->ts_f1 : s == 1 ? &q->ts_f2 : s == 2 ? &q->ts_b3 : &q->ts_b4;
    *t = g.ts[s];
    if (s == 3) {
      const int groups = std::min(g.b4_groups_cap[k], ceil_div(q->chunk_psf, g.b4_psfs));
      q->b4_gsize = ceil_div(q->chunk_psf, groups);
      q->b4_groups_max = ceil_div(q->chunk_psf, q->b4_gsize);
      q->b4_ksplit_tuned = b4_split_for(q, g.b4_ks);
      derive_tiles(q, q->b4_ksplit_tuned);
    }
  }
}

GemmArgs group_stage_args(dlx_plan* q, int s) {
  switch (s) {
    case 0: return args_f1(q, 0, q->F);
    case 1: return args_f2(q, 0, q->F);
    case 2: return args_b3(q, 0, q->F, nullptr);
    default: return args_b4(q, 0, 0, q->F);
  }
}

// Block table of a grouped GEMM launch, in dispatch order. Workgroup g goes to XCD g mod 8 and each
// XCD takes its workgroups in order, so the table is laid out as eight queues, entry j of queue x at
// position 8 j + x. Every problem's logical workgroups are cut into eight contiguous ranges whose
// sizes differ by at most one, one range per queue: each XCD then gets an equal share of every
// problem (tiles differ in depth from problem to problem, not within one), and the tiles of a range,
// which share operands, stay on one L2. The ranges that take a problem's remainder start at the
// first queue that is one entry short, so queue x always ends with ceil((n - x) / 8) entries.
// Returns an empty table if that count does not hold (not expected).
std::vector<int2> xcd_queue_table(const std::vector<std::pair<int, int>>& problem_wgs) {
  constexpr int kXcds = 8;
  std::vector<int2> q[kXcds];
  long long n = 0;
  for (const auto& pw : problem_wgs) {
    const int nw = pw.second, base = nw / kXcds, extra = nw % kXcds;
    const int start = (int)(n % kXcds);
    int w = 0;
    for (int j = 0; j < kXcds; ++j) {
      const int x = (start + j) % kXcds;
      const int cnt = base + (j < extra ? 1 : 0);
      for (int i = 0; i < cnt; ++i) q[x].push_back(make_int2(pw.first, w++));
    }
    n += nw;
  }
  std::vector<int2> tab((size_t)n);
  for (int x = 0; x < kXcds; ++x) {
    if ((long long)q[x].size() != (n - x + kXcds - 1) / kXcds) return {};
    for (size_t j = 0; j < q[x].size(); ++j) tab[j * kXcds + x] = q[x][j];
  }
  return tab;
}

// Arguments and block table of GEMM stage s for the current tiles, uploaded (problems in order of
// decreasing work, so the largest start first on every XCD).
hipError_t group_stage_upload(dlx_plan* p, int s) {
  GroupPlan& g = *p->group;
  group_apply_tiles(p, s);
  const int n = (int)p->subs.size();
  std::vector<GemmArgs> args(n);
  std::vector<std::pair<int, int>> wgs;
  long long n_wg = 0;
  for (int k : p->order) {
    GemmArgs a = group_stage_args(p->subs[k], s);
    a.sources = nullptr;
    a.src_off = p->offs[k].sources;
    args[k] = a;
    wgs.emplace_back(k, wg_count(a));
    n_wg += wg_count(a);
  }
  const std::vector<int2> tab = xcd_queue_table(wgs);
  if ((long long)tab.size() != n_wg || n_wg > g.cap_wg[s]) return hipErrorInvalidValue;
  hipError_t e = hipMemcpy(g.d_gargs[s], args.data(), sizeof(GemmArgs) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess && !tab.empty())
    e = hipMemcpy(g.d_gtab[s], tab.data(), sizeof(int2) * tab.size(), hipMemcpyHostToDevice);
  g.n_wg[s] = (int)tab.size();
  return e;
}

hipError_t group_gemm(dlx_plan* p, int s, const float* sources, hipStream_t st) {
  const GroupPlan& g = *p->group;
  return launch_gemm_group(kGroupKinds[s], p->bf16(), g.ts[s], g.d_gargs[s], g.d_gtab[s], g.n_wg[s], sources, st);
}

// Time every compiled tile shape of each stage (and B4's splits) as one grouped launch on the
// zeroed workspaces, keep the fastest.
hipError_t group_autotune(dlx_plan* p) {
  GroupPlan& g = *p->group;
  hipEvent_t t0, t1;
  hipError_t e = hipEventCreate(&t0);
  if (e != hipSuccess) return e;
  if ((e = hipEventCreate(&t1)) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return e;
  }
  const char* env = std::getenv("DLX_TUNE_LOG");
  const bool log = env && env[0] == '1';
  for (int s = 0; s < 4 && e == hipSuccess; ++s) {
    TileShape best = g.ts[s];
    int best_ks = g.b4_ks;
    float best_ms = 1e30f;
    const int n_ks = s == 3 ? 3 : 1;
    for (int ci = 0; ci < (int)(sizeof(kTileShapes) / sizeof(kTileShapes[0])) * n_ks && e == hipSuccess; ++ci) {
      const TileShape cand = kTileShapes[ci / n_ks];
      if (!tile_supported(kGroupKinds[s], p->bf16(), true, cand)) continue;
      g.ts[s] = cand;
      if (s == 3) g.b4_ks = 1 << (ci % n_ks);
      if ((e = group_stage_upload(p, s)) != hipSuccess) break;
      if ((e = group_gemm(p, s, g.d_tune_src, nullptr)) != hipSuccess) break;   // warm-up
      if ((e = hipEventRecord(t0, nullptr)) != hipSuccess) break;
      for (int r = 0; r < 2 && e == hipSuccess; ++r) e = group_gemm(p, s, g.d_tune_src, nullptr);
      if (e != hipSuccess) break;
      if ((e = hipEventRecord(t1, nullptr)) != hipSuccess) break;
      if ((e = hipEventSynchronize(t1)) != hipSuccess) break;
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
      if (log)
        std::fprintf(stderr, "dlx group tune: stage %d tile %dx%d ksplit %d: %.4f ms per launch\n", kGroupKinds[s],
                     cand.bm(), cand.bn(), g.b4_ks, ms / 2);
      if (ms < best_ms) {
        best_ms = ms;
        best = cand;
        best_ks = g.b4_ks;
      }
    }
    g.ts[s] = best;
    g.b4_ks = best_ks;
    if (s == 3 && e == hipSuccess) {   // then B4's PSFs per group, with its tile and split
      const int cands[4] = {8, 16, 32, 64};
      int best_gp = g.b4_psfs;
      best_ms = 1e30f;
      for (int gp : cands) {
        g.b4_psfs = gp;
        if ((e = group_stage_upload(p, s)) != hipSuccess) break;
        if ((e = group_gemm(p, s, g.d_tune_src, nullptr)) != hipSuccess) break;
        if ((e = hipEventRecord(t0, nullptr)) != hipSuccess) break;
        for (int r = 0; r < 2 && e == hipSuccess; ++r) e = group_gemm(p, s, g.d_tune_src, nullptr);
        if (e != hipSuccess) break;
        if ((e = hipEventRecord(t1, nullptr)) != hipSuccess) break;
        if ((e = hipEventSynchronize(t1)) != hipSuccess) break;
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
        if (log) std::fprintf(stderr, "dlx group tune: B4 %d PSFs per group: %.4f ms per launch\n", gp, ms / 2);
        if (ms < best_ms) {
          best_ms = ms;
          best_gp = gp;
        }
      }
      g.b4_psfs = best_gp;
    }
    if (e == hipSuccess) e = group_stage_upload(p, s);
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return e;
}

// Arguments and block tables of the small stages (after the tiles are final: the dL/dOPD reduction
// follows B4's groups and split).
hipError_t group_small_upload(dlx_plan* p) {
  GroupPlan& g = *p->group;
  const int n = (int)p->subs.size();
  std::vector<PrepArgs> prep(n);
  std::vector<PupilArgs> pupil(n);
  std::vector<BinLossArgs> bl(n);
  std::vector<GradArgs> grad(n);
  std::vector<GroupBlock> t_prep, t_pupil, t_bl[5], t_gopd, t_z, t_fin;
  for (int k : p->order) {
    const dlx_plan* q = p->subs[k];
    const dlx_offsets& o = p->offs[k];
    const long long npix = (long long)q->Ni * q->Ni;
    PrepArgs& a = prep[k];
    a.Nz = q->Nz;
    a.Ni = q->Ni;
    a.nb_opd = (int)((npix + 255) / 256);
    a.n_norm = q->n_norm_part;
    a.L = q->L;
    a.ldt = q->ldNi;
    a.npix = npix;
    a.n_tilt = (long long)q->n_psf * q->ldNi;
    a.tplane = a.n_tilt;
    a.opd = q->d_opd;
    a.norm_part = q->d_norm;
    a.wl = q->d_wl;
    a.x = q->d_x;
    a.tx = q->d_tx;
    a.ty = q->d_ty;
    a.o_trans = o.transmission;
    a.o_z = o.zernike_basis;
    a.o_c = o.zernike_coeffs;
    a.o_src = o.sources;
    const int nb_prep = a.nb_opd + a.n_norm + (int)((a.n_tilt + 255) / 256);
    for (int b = 0; b < nb_prep; ++b) t_prep.push_back(GroupBlock{k, b, 0, 0});

    PupilArgs& u = pupil[k];
    u.opd = q->d_opd;
    u.screen = q->d_screen;
    u.norm_part = q->d_norm;
    u.n_norm = q->n_norm_part;
    u.Ni = q->Ni;
    u.ldp = q->ldNi;
    u.h = q->hNi();
    u.wl = q->d_wl;
    u.P0T = q->d_P0T;
    u.plane = (long long)q->Ni * q->ldNi;
    u.by_wl = 2LL * q->Ni * q->ldNi;
    u.o_trans = o.transmission;
    u.L = q->L;
    for (int l = 0; l < q->L; l += kPupilGroupWl)
      for (int y = 0; y < (q->ldNi + 31) / 32; ++y)
        for (int x = 0; x < (q->Ni + 31) / 32; ++x) t_pupil.push_back(GroupBlock{k, x, y, l});

    BinLossArgs& b = bl[k];
    b.E = q->d_Y;
    b.plane = (long long)q->chunk_psf * q->No * q->ldNo;
    b.by_psf = (long long)q->No * q->ldNo;
    b.ld = q->ldNo;
    b.S = q->S;
    b.L = q->L;
    b.Q = q->Q;
    b.Nd = q->Nd;
    b.fh = q->hNo();
    b.fs = q->sNo();
    b.ldg = q->ldNo;
    b.nb = bin_loss_block_count((long long)q->Nd * q->Nd);
    b.wl = q->d_wl;
    b.kst = 0;
    b.g_by_frame = (long long)q->No * q->ldNo;
    b.bs = q->d_bs;
    b.blk = q->d_lossblk;
    b.status = q->d_status;
    b.G = q->d_G;
    b.flux = q->d_flux;
    b.o_src = o.sources;
    b.o_flat = o.flat;
    b.o_k = o.intrapixel;
    b.o_img = o.images;
    const int cls = bin_class(q->Q);
    for (int x = 0; x < b.nb; ++x) t_bl[cls].push_back(GroupBlock{k, x, 0, 0});

    GradArgs& r = grad[k];
    r.gpart = q->d_gpart;
    r.G = q->b4_groups_max * q->b4_ksplit;
    r.npix = npix;
    r.gopd = q->d_gopd;
    r.Nz = q->Nz;
    r.nchunks = q->Nz > 0 ? zproj_chunks(npix, q->Nz) : 1;
    r.zchunk = ((npix + r.nchunks - 1) / r.nchunks + 1023) / 1024 * 1024;
    r.zpart = q->d_zpart;
    r.flux = q->d_flux;
    r.flux_blocks = b.nb;
    r.tiles_b4 = q->tiles_b4 * q->b4_ksplit;
    r.L = q->L;
    r.FS = q->F * q->S;
    r.nloss = b.nb;
    r.pos = q->d_pos;
    r.lossblk = q->d_lossblk;
    r.o_z = o.zernike_basis;
    r.o_c = o.zernike_coeffs;
    r.o_src = o.sources;
    r.o_loss = o.loss;
    for (int x = 0; x < (int)((npix + 255) / 256); ++x) t_gopd.push_back(GroupBlock{k, x, 0, 0});
    if (q->Nz > 0)
      for (int y = 0; y < r.nchunks; ++y)
        for (int x = 0; x < (q->Nz + 7) / 8; ++x) t_z.push_back(GroupBlock{k, x, y, 0});
    for (int x = 0; x < q->Nz + r.FS + 1; ++x) t_fin.push_back(GroupBlock{k, x, 0, 0});
  }
  // one device buffer for all of it
  auto bytes = [](size_t n, size_t sz) { return (n * sz + 255) & ~size_t(255); };
  size_t total = bytes(n, sizeof(PrepArgs)) + bytes(n, sizeof(PupilArgs)) + bytes(n, sizeof(BinLossArgs)) +
                 bytes(n, sizeof(GradArgs)) + bytes(t_prep.size(), sizeof(GroupBlock)) +
                 bytes(t_pupil.size(), sizeof(GroupBlock)) + bytes(t_gopd.size(), sizeof(GroupBlock)) +
                 bytes(t_z.size(), sizeof(GroupBlock)) + bytes(t_fin.size(), sizeof(GroupBlock));
  for (int c = 0; c < 5; ++c) total += bytes(t_bl[c].size(), sizeof(GroupBlock));
  char* base = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&base), total);
  if (e != hipSuccess) return e;
  g.dmem_small = base;
  size_t off = 0;
  auto put = [&](const void* src, size_t nbytes) -> char* {
    char* d = base + off;
    off += (nbytes + 255) & ~size_t(255);
    if (nbytes && e == hipSuccess) e = hipMemcpy(d, src, nbytes, hipMemcpyHostToDevice);
    return d;
  };
  g.d_prep = reinterpret_cast<PrepArgs*>(put(prep.data(), n * sizeof(PrepArgs)));
  g.d_pupil = reinterpret_cast<PupilArgs*>(put(pupil.data(), n * sizeof(PupilArgs)));
  g.d_bl = reinterpret_cast<BinLossArgs*>(put(bl.data(), n * sizeof(BinLossArgs)));
  g.d_grad = reinterpret_cast<GradArgs*>(put(grad.data(), n * sizeof(GradArgs)));
  g.d_prep_tab = reinterpret_cast<GroupBlock*>(put(t_prep.data(), t_prep.size() * sizeof(GroupBlock)));
  g.d_pupil_tab = reinterpret_cast<GroupBlock*>(put(t_pupil.data(), t_pupil.size() * sizeof(GroupBlock)));
  g.d_gopd_tab = reinterpret_cast<GroupBlock*>(put(t_gopd.data(), t_gopd.size() * sizeof(GroupBlock)));
  g.d_z_tab = reinterpret_cast<GroupBlock*>(put(t_z.data(), t_z.size() * sizeof(GroupBlock)));
  g.d_fin_tab = reinterpret_cast<GroupBlock*>(put(t_fin.data(), t_fin.size() * sizeof(GroupBlock)));
  for (int c = 0; c < 5; ++c) {
    g.d_bl_tab[c] = reinterpret_cast<GroupBlock*>(put(t_bl[c].data(), t_bl[c].size() * sizeof(GroupBlock)));
    g.n_bl[c] = (int)t_bl[c].size();
  }
  g.n_prep = (int)t_prep.size();
  g.n_pupil = (int)t_pupil.size();
  g.n_gopd = (int)t_gopd.size();
  g.n_z = (int)t_z.size();
  g.n_fin = (int)t_fin.size();
  return e;
}

void group_free(GroupPlan* g) {
  if (!g) return;
  if (g->dmem) (void)hipFree(g->dmem);
  if (g->dmem_small) (void)hipFree(g->dmem_small);
  delete g;
}

// Build the grouped launches of a multi-problem plan whose sub-plans exist (created without
// tuning): device buffers for the GEMM arguments and tables (sized for the smallest tile and the
// largest B4 split), then the tiles (tuned unless `tune` is false), then the small stages.
dlx_status group_build(dlx_plan* p, bool tune) {
  for (const dlx_plan* q : p->subs)
    if (q->n_chunks != 1 || q->F != 1 || q->seed_pass || !q->fold || q->Nmap != 0 || q->dither) return DLX_OK;
  GroupPlan* g = new (std::nothrow) GroupPlan();
  if (!g) return DLX_ERR_OOM;
  p->group = g;
  const int n = (int)p->subs.size();
  const dlx_plan* q0 = p->subs[0];
  for (int s = 0; s < 4; ++s) g->ts[s] = s == 0 ? q0->ts_f1 : s == 1 ? q0->ts_f2 : s == 2 ? q0->ts_b3 : q0->ts_b4;
  g->b4_ks = 1;
  for (const dlx_plan* q : p->subs) g->b4_groups_cap.push_back(q->b4_groups_alloc);
  long long total_src = 0;
  for (int k = 0; k < n; ++k) {
    dlx_plan* q = p->subs[k];
    total_src = std::max<long long>(total_src, p->offs[k].sources + 3LL * q->F * q->S);
    const int fm = q->hNo(), fi = q->hNi();
    const int items = q->chunk_psf;
    g->cap_wg[0] += ceil_div(fm, 32) * ceil_div(q->Ni, 32) * items;
    g->cap_wg[1] += ceil_div(q->No, 32) * ceil_div(fm, 32) * items;
    g->cap_wg[2] += ceil_div(fi, 32) * ceil_div(q->No, 32) * items;
    g->cap_wg[3] += ceil_div(fi, 32) * ceil_div(q->Ni, 32) * q->b4_groups_alloc * 4;
  }
  size_t total = 0;
  auto bytes = [](size_t c, size_t sz) { return (c * sz + 255) & ~size_t(255); };
  for (int s = 0; s < 4; ++s) total += bytes(n, sizeof(GemmArgs)) + bytes(g->cap_wg[s], sizeof(int2));
  total += bytes(total_src, sizeof(float));
  if (hipMalloc(&g->dmem, total) != hipSuccess) {
    group_free(g);
    p->group = nullptr;
    return DLX_ERR_OOM;
  }
  char* c = static_cast<char*>(g->dmem);
  for (int s = 0; s < 4; ++s) {
    g->d_gargs[s] = reinterpret_cast<GemmArgs*>(c);
    c += bytes(n, sizeof(GemmArgs));
    g->d_gtab[s] = reinterpret_cast<int2*>(c);
    c += bytes(g->cap_wg[s], sizeof(int2));
  }
  g->d_tune_src = reinterpret_cast<float*>(c);
  hipError_t e = hipMemset(g->d_tune_src, 0, sizeof(float) * total_src);
  for (int s = 0; s < 4 && e == hipSuccess; ++s) e = group_stage_upload(p, s);
  if (e == hipSuccess && tune) e = group_autotune(p);
  if (e == hipSuccess) e = group_small_upload(p);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    group_free(g);
    p->group = nullptr;
    return DLX_ERR_HIP;
  }
  return DLX_OK;
}

// dlx_eval over every problem, one launch per stage.
dlx_status group_eval(dlx_plan* p, const dlx_eval_args* a, hipStream_t st) {
  const GroupPlan& g = *p->group;
  GroupCall call;
  call.transmission = a->transmission;
  call.zbasis = a->zernike_basis;
  call.coeffs = a->zernike_coeffs;
  call.sources = a->sources;
  call.flat = a->flat;
  call.intrapixel = a->intrapixel;
  call.data = a->data;
  call.binned = a->binned;
  call.model = a->model;
  call.r = a->dloss_dmodel;
  call.loss = a->loss;
  call.grad_flat = a->grad_flat;
  call.grad_zernike = a->grad_zernike;
  call.grad_sources = a->grad_sources;
  call.kind = (int)a->loss_kind;
  call.mu = a->prior_mu;
  call.inv_s2 = 1.0 / (a->prior_sigma * a->prior_sigma);
  for (dlx_plan* q : p->subs) q->fields_valid = false;
  {
    Stage sg(p, st, DLX_STAGE_PREP, p->n_psf);
    DLX_HIP(launch_prep_group(g.d_prep, g.d_prep_tab, g.n_prep, call, st));
    DLX_HIP(launch_pupil_group(g.d_pupil, g.d_pupil_tab, g.n_pupil, call, st));
  }
  {
    Stage sg(p, st, DLX_STAGE_F1, p->n_psf);
    DLX_HIP(group_gemm(p, 0, nullptr, st));
  }
  {
    Stage sg(p, st, DLX_STAGE_F2, p->n_psf);
    DLX_HIP(group_gemm(p, 1, nullptr, st));
  }
  {
    Stage sg(p, st, DLX_STAGE_BIN, p->n_psf);
    for (int c = 0; c < 5; ++c) DLX_HIP(launch_bin_loss_group(g.qt_of[c], g.d_bl, g.d_bl_tab[c], g.n_bl[c], call, st));
  }
  {
    Stage sg(p, st, DLX_STAGE_B3, p->n_psf);
    DLX_HIP(group_gemm(p, 2, a->sources, st));
  }
  {
    Stage sg(p, st, DLX_STAGE_B4, p->n_psf);
    DLX_HIP(group_gemm(p, 3, nullptr, st));
  }
  Stage sg(p, st, DLX_STAGE_GRAD, p->n_psf);
  DLX_HIP(launch_grad_group(g.d_grad, g.d_gopd_tab, g.n_gopd, g.d_z_tab, g.n_z, g.d_fin_tab, g.n_fin, call, st));
  return DLX_OK;
}

constexpr int kSideStreams = 4;

// One plan per problem; problem k's arrays sit at offs[k] in every packed array.
dlx_status create_multi(const dlx_problem_desc* probs, int32_t n, dlx_precision prec, int32_t flags, size_t limit,
                        dlx_plan** out) {
  dlx_plan* p = new (std::nothrow) dlx_plan();
  if (!p) return DLX_ERR_OOM;
  p->prec = prec;
  p->n_psf = 0;
  // grouped launches tune the shared tiles over all problems at once: the sub-plans skip their own
  const bool grouped = group_eligible(probs, n, flags);
  const bool tune = !(flags & DLX_FLAG_NO_AUTOTUNE);
  dlx_offsets o{};
  for (int k = 0; k < n; ++k) {
    dlx_plan* sub = nullptr;
    const dlx_status s = dlx_plan_create(&probs[k], 1, prec, grouped ? (flags | DLX_FLAG_NO_AUTOTUNE) : flags, limit,
                                         &sub);
    if (s != DLX_OK) {
      dlx_plan_destroy(p);
      return s;
    }
    p->subs.push_back(sub);
    p->offs.push_back(o);
    p->pool_bytes += sub->pool_bytes;
    p->n_psf += sub->n_psf;
    const dlx_problem_desc& d = probs[k];
    const long long ni2 = (long long)d.n_pupil * d.n_pupil, nd = d.n_focal / d.oversample;
    o.transmission += ni2;
    o.zernike_basis += (long long)d.n_zernike * ni2;
    o.map_basis += (long long)d.n_pupil * d.n_map;
    o.zernike_coeffs += d.n_zernike;
    o.phase_map += (long long)d.n_map * d.n_map;
    o.sources += 3LL * (d.frame_dithers ? 1 : d.n_frames) * d.n_sources;
    o.flat += nd * nd;
    o.intrapixel += (long long)d.oversample * d.oversample * ((flags & DLX_FLAG_PIXEL_KERNEL) ? nd * nd : 1);
    o.images += (long long)d.n_frames * nd * nd;
    o.loss += 1;
  }
  // Longest-processing-time assignment: problems by MFT work, largest first, each to the
  // side stream with the least work so far.
  std::vector<double> cost(n), load(kSideStreams, 0.0);
  for (int k = 0; k < n; ++k) {
    const dlx_plan* q = p->subs[k];
    cost[k] = (double)q->n_psf * q->No * q->Ni * (double)(q->Ni + q->No);
  }
  p->order.resize(n);
  for (int k = 0; k < n; ++k) p->order[k] = k;
  std::stable_sort(p->order.begin(), p->order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  p->lane.assign(n, 0);
  for (int k : p->order) {
    const int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    p->lane[k] = s;
    load[s] += cost[k];
  }
  p->side.resize(kSideStreams, nullptr);
  p->joins.resize(kSideStreams, nullptr);
  bool ok = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < kSideStreams; ++i) {
    ok = hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&p->joins[i], hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    dlx_plan_destroy(p);
    return DLX_ERR_HIP;
  }
  if (grouped) {
    dlx_status s = group_build(p, tune);
    if (s == DLX_OK && !p->group && tune) {   // a problem needs more than one chunk: tune each on its own
      for (dlx_plan* q : p->subs) {
        if (autotune_cached(q) != hipSuccess || hipMemset(q->d_status, 0, sizeof(int)) != hipSuccess) {
          s = DLX_ERR_HIP;
          break;
        }
      }
      if (s == DLX_OK && hipDeviceSynchronize() != hipSuccess) s = DLX_ERR_HIP;
    }
    if (s != DLX_OK) {
      dlx_plan_destroy(p);
      return s;
    }
  }
  *out = p;
  return DLX_OK;
}

// Run fn(k, sub, stream) for every problem, spread over the side streams
// (balanced by MFT work), ordered after prior work on `st` and joined back
// into `st` (also under stream capture, where it records parallel branches).
template <class Fn>
dlx_status run_multi(dlx_plan* p, hipStream_t st, Fn fn) {
  DLX_HIP(hipEventRecord(p->fork, st));
  for (hipStream_t s : p->side) DLX_HIP(hipStreamWaitEvent(s, p->fork, 0));
  dlx_status status = DLX_OK;
  for (size_t i = 0; i < p->order.size() && status == DLX_OK; ++i) {
    const int k = p->order[i];
    status = fn(k, p->subs[k], p->side[p->lane[k]]);
  }
  for (size_t i = 0; i < p->side.size(); ++i) {
    DLX_HIP(hipEventRecord(p->joins[i], p->side[i]));
    DLX_HIP(hipStreamWaitEvent(st, p->joins[i], 0));
  }
  return status;
}

template <class T>
T* at(T* base, long long off) {
  return base ? base + off : nullptr;
}

}  // namespace

extern "C" {

dlx_status dlx_plan_create(const dlx_problem_desc* probs, int32_t n_probs, dlx_precision precision, int32_t flags,
                           size_t workspace_limit_bytes, dlx_plan** out) {
  if (!out) return DLX_ERR_INVALID_ARG;
  *out = nullptr;
  dlx_status v = dlx_validate(probs, n_probs);
  if (v != DLX_OK) return v;
  if (precision != DLX_FP32 && precision != DLX_BF16X3) return DLX_ERR_INVALID_ARG;
  if ((flags & ~(DLX_FLAG_NO_AUTOTUNE | DLX_FLAG_SEED_PASS | DLX_FLAG_STORE_FIELDS | DLX_FLAG_PIXEL_KERNEL |
                 DLX_FLAG_DENSE_MFT | DLX_FLAG_GROUPED)) != 0)
    return DLX_ERR_INVALID_ARG;
  if (n_probs > 1) return create_multi(probs, n_probs, precision, flags, workspace_limit_bytes, out);
  const dlx_problem_desc& d = probs[0];

  dlx_plan* p = new (std::nothrow) dlx_plan();
  if (!p) return DLX_ERR_OOM;
  p->Ni = d.n_pupil;
  p->No = d.n_focal;
  p->Q = d.oversample;
  p->Nd = d.n_focal / d.oversample;
  p->L = d.n_wavelengths;
  p->S = d.n_sources;
  p->F = d.n_frames;
  p->F_img = d.n_frames;
  p->Nd_img = p->Nd;
  if (d.frame_dithers) {  // one enlarged frame for the MFT stages; the images are its windows
    p->dither = true;
    p->margin = d.dither_margin;
    p->Nd = p->Nd_img + 2 * p->margin;
    p->No = p->Q * p->Nd;
    p->F = 1;
    p->win.resize(2 * (size_t)p->F_img);
    for (int f = 0; f < p->F_img; ++f) {
      p->win[2 * f] = p->margin - d.frame_dithers[2 * f + 1];
      p->win[2 * f + 1] = p->margin - d.frame_dithers[2 * f];
    }
  }
  p->Nz = d.n_zernike;
  p->Nmap = d.n_map;
  p->D = d.diameter_m;
  p->du = d.focal_pixel_rad;
  p->dx = d.diameter_m / d.n_pupil;
  p->lam.assign(d.wavelengths_m, d.wavelengths_m + d.n_wavelengths);
  p->wts.assign(d.spectral_weights, d.spectral_weights + d.n_wavelengths);
  p->prec = precision;
  p->ldNi = round_up(p->Ni, 16);
  p->ldNo = round_up(p->No, 16);
  p->fold = (flags & DLX_FLAG_DENSE_MFT) == 0;
  p->n_psf = p->F * p->S * p->L;

  // chunk of whole frames whose intermediates fit the budget (stored fields: every frame in one chunk)
  p->store_fields = (flags & DLX_FLAG_STORE_FIELDS) != 0;
  p->k_per_pixel = (flags & DLX_FLAG_PIXEL_KERNEL) != 0;
  if (p->k_per_pixel && p->dither) {   // the windows would need a frame-dependent binning
    delete p;
    return DLX_ERR_UNSUPPORTED;
  }
  size_t budget = workspace_limit_bytes ? workspace_limit_bytes : kDefaultChunkBudget;
  if (p->store_fields && !workspace_limit_bytes) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete p;
      return DLX_ERR_HIP;
    }
    budget = free_b / 10 * 8;
  }
  const size_t psf_bytes = per_psf_bytes(p);
  const size_t frame_bytes = psf_bytes * p->S * p->L + per_frame_bytes(p);
  const size_t fixed = sizeof(float) * 2 * (size_t)p->L *
                       ((size_t)p->No * p->ldNi + (size_t)p->Ni * p->ldNo + (size_t)p->Ni * p->ldNi);
  if (workspace_limit_bytes) {
    if (fixed + frame_bytes > budget) {
      delete p;
      return DLX_ERR_OOM;
    }
    budget -= fixed;
  }
  p->frames_per_chunk = (int)std::max<size_t>(1, std::min<size_t>(p->F, budget / frame_bytes));
  if (p->store_fields && p->frames_per_chunk < p->F) {
    delete p;
    return DLX_ERR_OOM;
  }
  p->n_chunks = ceil_div(p->F, p->frames_per_chunk);
  p->chunk_psf = p->frames_per_chunk * p->S * p->L;

  // tiles
  const bool fo = p->fold;
  const int mNo = fo ? p->hNo() : p->No, mNi = fo ? p->hNi() : p->Ni;   // folded DFT-side sizes
  p->ts_f1 = choose_tile(mNo, p->Ni, p->chunk_psf, 1, fo);
  p->ts_b3 = choose_tile(mNi, p->No, p->chunk_psf, 1, fo);
  const int sl = p->S * p->L;
  p->ts_f2 = choose_tile(p->No, mNo, (long long)p->frames_per_chunk * sl, 1, fo);
  {
    const int t = ceil_div(mNi, 128) * ceil_div(p->Ni, 128);
    const int g = std::max(1, std::min(ceil_div(kTargetWG, t), p->chunk_psf));
    p->b4_gsize = ceil_div(p->chunk_psf, g);
    p->b4_groups_max = ceil_div(p->chunk_psf, p->b4_gsize);
    p->ts_b4 = choose_tile(mNi, p->Ni, p->b4_groups_max, 1, fo);
    // the autotuner also tries twice and four times this group size (fewer partial planes to write
    // and add up, fewer workgroups); the partial planes are sized for this one, the most groups
    p->b4_gsize_default = p->b4_gsize;
    p->b4_groups_alloc = p->b4_groups_max;
  }
  derive_tiles(p);
  // partial-sum buffers are sized for the smallest candidate tile (32 x 32) and the largest split
  p->tiles_b4_cap = ceil_div(p->Ni, 32) * ceil_div(p->Ni, 32);
  p->ksplit_cap = 4;
  p->loss_blocks = loss_block_count((long long)p->Nd_img * p->Nd_img);
  p->seed_blocks = seed_block_count((long long)p->Nd * p->Nd);
  // the dense B3 streams a frame's G slower than a separate pass once G outgrows an XCD's L2; the
  // folded B3 (a quarter of the matrix work per G element read) does not, up to frames of 2048^2
  // focal samples (16.8 MB of G)
  p->seed_pass = (flags & DLX_FLAG_SEED_PASS) ||
                 (!p->fold && sizeof(float) * (size_t)p->No * p->ldNo > kSeedFuseMaxBytes);
  {
    const long long npix = (long long)p->Ni * p->Ni;
    p->n_norm_part = (int)std::max<long long>(1, std::min<long long>(256, (npix + 4095) / 4096));
  }

  Pool sizing{nullptr, 0};
  layout(p, sizing);
  p->pool_bytes = sizing.off + 256;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    delete p;
    return DLX_ERR_HIP;
  }
  if (p->pool_bytes > free_b) {
    delete p;
    return DLX_ERR_OOM;
  }
  if (hipMalloc(&p->pool, p->pool_bytes) != hipSuccess) {
    delete p;
    return DLX_ERR_OOM;
  }
  Pool pool{reinterpret_cast<char*>(p->pool), 0};
  layout(p, pool);

  std::vector<WlInfo> wl(p->L);
  for (int l = 0; l < p->L; ++l) {
    wl[l].lam = p->lam[l];
    wl[l].w = (float)p->wts[l];
    wl[l].scale = (float)(p->dx * p->du / p->lam[l]);
    wl[l].kphase = (float)(kTwoPi / p->lam[l]);
    wl[l].pad = 0.f;
  }
  hipError_t e = hipMemset(p->pool, 0, p->pool_bytes);
  if (e == hipSuccess) e = hipMemcpy(p->d_wl, wl.data(), sizeof(WlInfo) * p->L, hipMemcpyHostToDevice);
  if (e == hipSuccess && p->dither)
    e = hipMemcpy(p->d_win, p->win.data(), sizeof(int) * p->win.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_dft(p, nullptr);
  if (e == hipSuccess && !(flags & DLX_FLAG_NO_AUTOTUNE)) e = autotune_cached(p);
  if (e == hipSuccess) e = hipMemset(p->d_status, 0, sizeof(int));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(p->pool);
    delete p;
    return DLX_ERR_HIP;
  }
  *out = p;
  return DLX_OK;
}

dlx_status dlx_plan_destroy(dlx_plan* p) {
  if (!p) return DLX_OK;
  if (p->multi() || !p->side.empty()) {
    dlx_status s = DLX_OK;
    if (hipDeviceSynchronize() != hipSuccess) s = DLX_ERR_HIP;
    group_free(p->group);
    p->group = nullptr;
    for (hipEvent_t ev : p->ev_pool) (void)hipEventDestroy(ev);
    for (dlx_plan* sub : p->subs)
      if (dlx_plan_destroy(sub) != DLX_OK) s = DLX_ERR_HIP;
    for (hipStream_t st : p->side)
      if (st) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : p->joins)
      if (ev) (void)hipEventDestroy(ev);
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    delete p;
    return s;
  }
  const hipError_t e1 = hipDeviceSynchronize();
  for (hipEvent_t ev : p->ev_pool) (void)hipEventDestroy(ev);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  const hipError_t e2 = p->pool ? hipFree(p->pool) : hipSuccess;
  delete p;
  return (e1 == hipSuccess && e2 == hipSuccess) ? DLX_OK : DLX_ERR_HIP;
}

size_t dlx_plan_workspace_bytes(const dlx_plan* p) { return p ? p->pool_bytes : 0; }

dlx_status dlx_plan_offsets(const dlx_plan* p, int32_t k, dlx_offsets* out) {
  if (!p || !out) return DLX_ERR_INVALID_ARG;
  if (!p->multi()) {
    if (k != 0) return DLX_ERR_INVALID_ARG;
    *out = dlx_offsets{};
    return DLX_OK;
  }
  if (k < 0 || k >= (int32_t)p->subs.size()) return DLX_ERR_INVALID_ARG;
  *out = p->offs[k];
  return DLX_OK;
}

int32_t dlx_plan_problems(const dlx_plan* p) { return p ? (p->multi() ? (int32_t)p->subs.size() : 1) : 0; }

dlx_status dlx_plan_tiles(const dlx_plan* p, int32_t* tiles) {
  if (!p || !tiles) return DLX_ERR_INVALID_ARG;
  if (p->multi()) return dlx_plan_tiles(p->subs[0], tiles);
  const TileShape t[4] = {p->ts_f1, p->ts_f2, p->ts_b3, p->ts_b4};
  for (int k = 0; k < 4; ++k) {
    tiles[2 * k] = t[k].wm;
    tiles[2 * k + 1] = t[k].wn;
  }
  return DLX_OK;
}

dlx_status dlx_plan_profile(dlx_plan* p, int32_t enable) {
  if (!p) return DLX_ERR_INVALID_ARG;
  if (p->multi()) {
    for (dlx_plan* sub : p->subs) {
      const dlx_status s = dlx_plan_profile(sub, enable);
      if (s != DLX_OK) return s;
    }
    if (!p->group) return DLX_OK;   // grouped launches record their stages on the plan itself
  }
  if (enable && p->ev_pool.empty()) {
    p->ev_pool.resize(kEventPool);
    for (auto& ev : p->ev_pool) DLX_HIP(hipEventCreate(&ev));
  }
  if (!enable) {
    p->recs.clear();
    p->ev_used = 0;
  }
  p->profiling = enable != 0;
  for (int i = 0; i < DLX_N_STAGES; ++i) {
    p->stage_ms[i] = 0.0;
    p->stage_launches[i] = 0;
    p->stage_psfs[i] = 0;
  }
  return DLX_OK;
}

dlx_status dlx_plan_stage_times(dlx_plan* p, double* total_ms, int64_t* launches, int64_t* psfs) {
  if (!p || !total_ms || !launches || !psfs) return DLX_ERR_INVALID_ARG;
  if (p->multi()) {  // summed over problems (they run concurrently on side streams)
    for (int i = 0; i < DLX_N_STAGES; ++i) {
      total_ms[i] = 0.0;
      launches[i] = psfs[i] = 0;
    }
    for (dlx_plan* sub : p->subs) {
      double ms[DLX_N_STAGES];
      int64_t la[DLX_N_STAGES], ps[DLX_N_STAGES];
      const dlx_status s = dlx_plan_stage_times(sub, ms, la, ps);
      if (s != DLX_OK) return s;
      for (int i = 0; i < DLX_N_STAGES; ++i) {
        total_ms[i] += ms[i];
        launches[i] += la[i];
        psfs[i] += ps[i];
      }
    }
    if (p->group) {   // the grouped launches' own stages
      DLX_HIP(flush_records(p));
      for (int i = 0; i < DLX_N_STAGES; ++i) {
        total_ms[i] += p->stage_ms[i];
        launches[i] += p->stage_launches[i];
        psfs[i] += p->stage_psfs[i];
        p->stage_ms[i] = 0.0;
        p->stage_launches[i] = 0;
        p->stage_psfs[i] = 0;
      }
    }
    return DLX_OK;
  }
  DLX_HIP(flush_records(p));
  for (int i = 0; i < DLX_N_STAGES; ++i) {
    total_ms[i] = p->stage_ms[i];
    launches[i] = p->stage_launches[i];
    psfs[i] = p->stage_psfs[i];
    p->stage_ms[i] = 0.0;
    p->stage_launches[i] = 0;
    p->stage_psfs[i] = 0;
  }
  return DLX_OK;
}

dlx_status dlx_plan_set_phase_screen(dlx_plan* p, int32_t problem, const float* screen, void* stream) {
  if (!p) return DLX_ERR_INVALID_ARG;
  if (p->multi()) {
    if (problem < 0 || problem >= (int32_t)p->subs.size()) return DLX_ERR_INVALID_ARG;
    return dlx_plan_set_phase_screen(p->subs[problem], 0, screen, stream);
  }
  if (problem != 0) return DLX_ERR_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const long long n = (long long)p->Ni * p->Ni;
  if (screen) {
    DLX_HIP(hipMemcpyAsync(p->d_screen, screen, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
  } else {
    DLX_HIP(launch_zero(p->d_screen, n, st));
  }
  return DLX_OK;
}

dlx_status dlx_plan_sync(dlx_plan* p, void* stream) {
  if (!p) return DLX_ERR_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (p->multi()) {
    DLX_HIP(hipStreamSynchronize(st));
    dlx_status worst = DLX_OK;
    for (dlx_plan* sub : p->subs) {
      const dlx_status s = dlx_plan_sync(sub, stream);
      if (s == DLX_ERR_HIP) return s;
      if (s == DLX_ERR_NONFINITE || (s == DLX_ERR_DOMAIN && worst == DLX_OK)) worst = s;
    }
    return worst;
  }
  DLX_HIP(hipStreamSynchronize(st));
  int h = 0;
  DLX_HIP(hipMemcpy(&h, p->d_status, sizeof(int), hipMemcpyDeviceToHost));
  DLX_HIP(hipMemset(p->d_status, 0, sizeof(int)));
  if (h & 1) return DLX_ERR_NONFINITE;
  if (h & 2) return DLX_ERR_DOMAIN;
  return DLX_OK;
}

dlx_status dlx_psf_forward(dlx_plan* p, const float* transmission, const float* zernike_basis,
                           const float* map_basis, const float* zernike_coeffs, const float* phase_map,
                           const float* sources, const float* flat, const float* intrapixel, float* binned_out,
                           float* model_out, void* stream) {
  if (!p || !ok_ptr(transmission) || !ok_ptr(sources) || !ok_ptr(flat) || !ok_ptr(binned_out) || !ok_ptr(model_out))
    return DLX_ERR_INVALID_ARG;
  if (p->multi()) {
    return run_multi(p, reinterpret_cast<hipStream_t>(stream), [&](int k, dlx_plan* q, hipStream_t s) {
      const dlx_offsets& o = p->offs[k];
      return dlx_psf_forward(q, at(transmission, o.transmission), q->Nz ? at(zernike_basis, o.zernike_basis) : nullptr,
                             q->Nmap ? at(map_basis, o.map_basis) : nullptr,
                             q->Nz ? at(zernike_coeffs, o.zernike_coeffs) : nullptr,
                             q->Nmap ? at(phase_map, o.phase_map) : nullptr, at(sources, o.sources), at(flat, o.flat),
                             at(intrapixel, o.intrapixel), at(binned_out, o.images), at(model_out, o.images), s);
    });
  }
  if (p->Nz > 0 && (!zernike_basis || !zernike_coeffs)) return DLX_ERR_INVALID_ARG;
  if ((p->Nmap > 0) != (map_basis != nullptr) || (p->Nmap > 0) != (phase_map != nullptr)) return DLX_ERR_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  {
    Stage sg(p, st, DLX_STAGE_PREP, p->n_psf);
    DLX_HIP(launch_prep(p, transmission, zernike_basis, map_basis, zernike_coeffs, phase_map, sources, st));
  }
  for (int c = 0; c < p->n_chunks; ++c) {
    const int f0 = c * p->frames_per_chunk;
    const int nf = std::min(p->frames_per_chunk, p->F - f0);
    const int nc = nf * p->S * p->L;
    {
      Stage sg(p, st, DLX_STAGE_F1, nc);
      DLX_HIP(run_f1(p, f0, nf, st));
    }
    {
      Stage sg(p, st, DLX_STAGE_F2, nc);
      DLX_HIP(run_f2(p, f0, nf, st));
    }
    Stage sg(p, st, DLX_STAGE_BIN, nc);
    if (p->dither) {  // bin the enlarged plane once, then cut every frame's window
      DLX_HIP(launch_intensity(p, f0, nf, sources, intrapixel, nullptr, p->d_Bbig, nullptr, st));
      DLX_HIP(launch_window(p, flat, binned_out, model_out, st));
    } else {
      DLX_HIP(launch_intensity(p, f0, nf, sources, intrapixel, flat, binned_out, model_out, st));
    }
  }
  p->fields_valid = p->store_fields;   // one chunk: E, the pupil pieces and the binned images stay
  return DLX_OK;
}

dlx_status dlx_loss_grad(dlx_plan* p, const float* model, const float* binned, const float* data, const float* flat,
                         dlx_loss_kind kind, double prior_mu, double prior_sigma, double* loss_out,
                         float* dloss_dmodel, double* grad_flat, void* stream) {
  if (!p || !model || !binned || !data || !flat || !loss_out || !dloss_dmodel || !grad_flat)
    return DLX_ERR_INVALID_ARG;
  if (p->multi()) {
    return run_multi(p, reinterpret_cast<hipStream_t>(stream), [&](int k, dlx_plan* q, hipStream_t s) {
      const dlx_offsets& o = p->offs[k];
      return dlx_loss_grad(q, at(model, o.images), at(binned, o.images), at(data, o.images), at(flat, o.flat), kind, prior_mu,
                           prior_sigma, at(loss_out, o.loss), at(dloss_dmodel, o.images), at(grad_flat, o.flat), s);
    });
  }
  if (kind != DLX_LOSS_POISSON && kind != DLX_LOSS_CHI2) return DLX_ERR_INVALID_ARG;
  if (!(prior_sigma > 0.0) || !std::isfinite(prior_sigma) || !std::isfinite(prior_mu)) return DLX_ERR_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Stage sg(p, st, DLX_STAGE_LOSS, p->n_psf);
  DLX_HIP(launch_loss(p, 0, p->F_img, 0, model, binned, data, flat, (int)kind, prior_mu, prior_sigma, dloss_dmodel,
                      grad_flat, nullptr, st));
  DLX_HIP(launch_loss_final(p, 1, loss_out, st));
  return DLX_OK;
}

dlx_status dlx_psf_backward(dlx_plan* p, const float* transmission, const float* zernike_basis,
                            const float* map_basis, const float* zernike_coeffs, const float* phase_map,
                            const float* sources, const float* flat, const float* intrapixel,
                            const float* dloss_dmodel, double* grad_zernike, double* grad_map, double* grad_sources,
                            double* grad_intrapixel, void* stream) {
  if (!p || !transmission || !sources || !flat || !dloss_dmodel || !grad_sources) return DLX_ERR_INVALID_ARG;
  if (p->multi()) {
    return run_multi(p, reinterpret_cast<hipStream_t>(stream), [&](int k, dlx_plan* q, hipStream_t s) {
      const dlx_offsets& o = p->offs[k];
      return dlx_psf_backward(q, at(transmission, o.transmission), q->Nz ? at(zernike_basis, o.zernike_basis) : nullptr,
                              q->Nmap ? at(map_basis, o.map_basis) : nullptr,
                              q->Nz ? at(zernike_coeffs, o.zernike_coeffs) : nullptr,
                              q->Nmap ? at(phase_map, o.phase_map) : nullptr, at(sources, o.sources), at(flat, o.flat),
                              at(intrapixel, o.intrapixel), at(dloss_dmodel, o.images),
                              q->Nz ? at(grad_zernike, o.zernike_coeffs) : nullptr,
                              q->Nmap ? at(grad_map, o.phase_map) : nullptr, at(grad_sources, o.sources),
                              at(grad_intrapixel, o.intrapixel), s);
    });
  }
  if (p->Nz > 0 && (!zernike_basis || !zernike_coeffs || !grad_zernike)) return DLX_ERR_INVALID_ARG;
  if (grad_intrapixel && p->Q > kMaxKgradQ) return DLX_ERR_UNSUPPORTED;
  if ((p->Nmap > 0) != (map_basis != nullptr) || (p->Nmap > 0) != (phase_map != nullptr) ||
      (p->Nmap > 0) != (grad_map != nullptr))
    return DLX_ERR_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // stored fields: the preceding forward left the pupil pieces, E and the per-star binned
  // images of every PSF in the workspace (one chunk); only the adjoint runs
  const bool reuse = p->store_fields && p->fields_valid;
  p->fields_valid = false;
  if (!reuse) {
    Stage sg(p, st, DLX_STAGE_PREP, p->n_psf);
    DLX_HIP(launch_prep(p, transmission, zernike_basis, map_basis, zernike_coeffs, phase_map, sources, st));
  }
  for (int c = 0; c < p->n_chunks; ++c) {
    const int f0 = c * p->frames_per_chunk;
    const int nf = std::min(p->frames_per_chunk, p->F - f0);
    const int nc = nf * p->S * p->L;
    if (!reuse) {
      {
        Stage sg(p, st, DLX_STAGE_F1, nc);
        DLX_HIP(run_f1(p, f0, nf, st));
      }
      {
        Stage sg(p, st, DLX_STAGE_F2, nc);
        DLX_HIP(run_f2(p, f0, nf, st));
      }
      {  // per-source binned images only (for the flux gradient)
        Stage sg(p, st, DLX_STAGE_BIN, nc);
        DLX_HIP(launch_intensity(p, f0, nf, sources, intrapixel, flat, nullptr, nullptr, st));
      }
    }
    {
      Stage sg(p, st, DLX_STAGE_SEED, nc);
      if (p->dither)
        DLX_HIP(launch_seed_gather(p, flat, dloss_dmodel, intrapixel, st));
      else
        DLX_HIP(launch_seed(p, f0, nf, flat, dloss_dmodel, intrapixel, st));
      if (grad_intrapixel) DLX_HIP(launch_kgrad(p, f0, nf, sources, flat, dloss_dmodel, grad_intrapixel, st));
      if (p->seed_pass) DLX_HIP(launch_seed_apply(p, f0, nf, sources, st));
    }
    DLX_HIP(run_adjoint(p, c, f0, nf, sources, st));
  }
  Stage sg(p, st, DLX_STAGE_GRAD, p->n_psf);
  DLX_HIP(launch_grad_reduce(p, zernike_basis, map_basis, grad_zernike, grad_map, grad_sources, nullptr, 0,
                             grad_intrapixel, st));
  return DLX_OK;
}

// Value and gradient, fused per chunk of frames: a frame's residual depends
// only on that frame's model, so each chunk runs forward, loss and adjoint
// back to back and the focal fields E of F2 are reused for the adjoint seed
// instead of being recomputed (2 MFTs per PSF instead of 3; memory stays one
// chunk of fields).
dlx_status dlx_eval(dlx_plan* p, const dlx_eval_args* a, void* stream) {
  if (!p || !a) return DLX_ERR_INVALID_ARG;
  if (p->multi()) {
    if (!a->transmission || !a->sources || !a->flat || !a->data || !a->binned || !a->model || !a->dloss_dmodel ||
        !a->loss || !a->grad_flat || !a->grad_sources)
      return DLX_ERR_INVALID_ARG;
    if (a->loss_kind != DLX_LOSS_POISSON && a->loss_kind != DLX_LOSS_CHI2) return DLX_ERR_INVALID_ARG;
    if (!(a->prior_sigma > 0.0) || !std::isfinite(a->prior_sigma) || !std::isfinite(a->prior_mu))
      return DLX_ERR_INVALID_ARG;
    if (p->group && !a->grad_intrapixel) {
      bool zok = true;   // every problem with Zernike terms needs the basis, coefficients and gradient
      for (const dlx_plan* q : p->subs) zok = zok && (q->Nz == 0 || (a->zernike_basis && a->zernike_coeffs && a->grad_zernike));
      if (!zok) return DLX_ERR_INVALID_ARG;
      return group_eval(p, a, reinterpret_cast<hipStream_t>(stream));
    }
    return run_multi(p, reinterpret_cast<hipStream_t>(stream), [&](int k, dlx_plan* q, hipStream_t s) {
      const dlx_offsets& o = p->offs[k];
      dlx_eval_args b = *a;
      b.transmission = at(a->transmission, o.transmission);
      b.zernike_basis = q->Nz ? at(a->zernike_basis, o.zernike_basis) : nullptr;
      b.map_basis = q->Nmap ? at(a->map_basis, o.map_basis) : nullptr;
      b.zernike_coeffs = q->Nz ? at(a->zernike_coeffs, o.zernike_coeffs) : nullptr;
      b.phase_map = q->Nmap ? at(a->phase_map, o.phase_map) : nullptr;
      b.sources = at(a->sources, o.sources);
      b.flat = at(a->flat, o.flat);
      b.intrapixel = at(a->intrapixel, o.intrapixel);
      b.data = at(a->data, o.images);
      b.binned = at(a->binned, o.images);
      b.model = at(a->model, o.images);
      b.dloss_dmodel = at(a->dloss_dmodel, o.images);
      b.loss = at(a->loss, o.loss);
      b.grad_flat = at(a->grad_flat, o.flat);
      b.grad_zernike = q->Nz ? at(a->grad_zernike, o.zernike_coeffs) : nullptr;
      b.grad_map = q->Nmap ? at(a->grad_map, o.phase_map) : nullptr;
      b.grad_sources = at(a->grad_sources, o.sources);
      b.grad_intrapixel = at(a->grad_intrapixel, o.intrapixel);
      return dlx_eval(q, &b, s);
    });
  }
  if (!a->transmission || !a->sources || !a->flat || !a->data || !a->binned || !a->model || !a->dloss_dmodel ||
      !a->loss || !a->grad_flat || !a->grad_sources)
    return DLX_ERR_INVALID_ARG;
  if (p->Nz > 0 && (!a->zernike_basis || !a->zernike_coeffs || !a->grad_zernike)) return DLX_ERR_INVALID_ARG;
  if ((p->Nmap > 0) != (a->map_basis != nullptr) || (p->Nmap > 0) != (a->phase_map != nullptr) ||
      (p->Nmap > 0) != (a->grad_map != nullptr))
    return DLX_ERR_INVALID_ARG;
  if (a->loss_kind != DLX_LOSS_POISSON && a->loss_kind != DLX_LOSS_CHI2) return DLX_ERR_INVALID_ARG;
  if (a->grad_intrapixel && p->Q > kMaxKgradQ) return DLX_ERR_UNSUPPORTED;
  if (!(a->prior_sigma > 0.0) || !std::isfinite(a->prior_sigma) || !std::isfinite(a->prior_mu))
    return DLX_ERR_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  p->fields_valid = false;
  {
    Stage sg(p, st, DLX_STAGE_PREP, p->n_psf);
    DLX_HIP(launch_prep(p, a->transmission, a->zernike_basis, a->map_basis, a->zernike_coeffs, a->phase_map,
                        a->sources, st));
  }
  for (int c = 0; c < p->n_chunks; ++c) {
    const int f0 = c * p->frames_per_chunk;
    const int nf = std::min(p->frames_per_chunk, p->F - f0);
    const int nc = nf * p->S * p->L;
    {
      Stage sg(p, st, DLX_STAGE_F1, nc);
      DLX_HIP(run_f1(p, f0, nf, st));
    }
    {
      Stage sg(p, st, DLX_STAGE_F2, nc);
      DLX_HIP(run_f2(p, f0, nf, st));
    }
    if (p->dither) {
      {  // the enlarged plane once, then every frame's window
        Stage sg(p, st, DLX_STAGE_BIN, nc);
        DLX_HIP(launch_intensity(p, f0, nf, a->sources, a->intrapixel, nullptr, p->d_Bbig, nullptr, st));
        DLX_HIP(launch_window(p, a->flat, a->binned, a->model, st));
      }
      {
        Stage sg(p, st, DLX_STAGE_LOSS, nc);
        DLX_HIP(launch_loss(p, 0, p->F_img, c, a->model, a->binned, a->data, a->flat, (int)a->loss_kind,
                            a->prior_mu, a->prior_sigma, a->dloss_dmodel, a->grad_flat, nullptr, st));
      }
      Stage sg(p, st, DLX_STAGE_SEED, nc);
      DLX_HIP(launch_seed_gather(p, a->flat, a->dloss_dmodel, a->intrapixel, st));
      if (a->grad_intrapixel) DLX_HIP(launch_kgrad(p, f0, nf, a->sources, a->flat, a->dloss_dmodel, a->grad_intrapixel, st));
      if (p->seed_pass) DLX_HIP(launch_seed_apply(p, f0, nf, a->sources, st));
    } else {
      if (p->frames_per_chunk == 1) {
        // one frame per chunk: binning, model, loss, residual, seed weights and flux partials in one
        // pass (with several frames per chunk the frames would serialise inside each block)
        Stage sg(p, st, DLX_STAGE_BIN, nc);
        DLX_HIP(launch_bin_loss(p, f0, nf, c, a->sources, a->intrapixel, a->flat, a->data, (int)a->loss_kind,
                                a->prior_mu, a->prior_sigma, a->binned, a->model, a->dloss_dmodel, a->grad_flat, st));
      } else {
        {
          Stage sg(p, st, DLX_STAGE_BIN, nc);
          DLX_HIP(launch_intensity(p, f0, nf, a->sources, a->intrapixel, a->flat, a->binned, a->model, st));
        }
        // loss, residual and the adjoint seed weights in one pass over the pixels
        Stage sg(p, st, DLX_STAGE_LOSS, nc);
        DLX_HIP(launch_loss(p, f0, nf, c, a->model, a->binned, a->data, a->flat, (int)a->loss_kind, a->prior_mu,
                            a->prior_sigma, a->dloss_dmodel, a->grad_flat, &a->intrapixel, st));
      }
      if (a->grad_intrapixel || p->seed_pass) {
        Stage sg(p, st, DLX_STAGE_SEED, nc);
        if (a->grad_intrapixel) DLX_HIP(launch_kgrad(p, f0, nf, a->sources, a->flat, a->dloss_dmodel, a->grad_intrapixel, st));
        if (p->seed_pass) DLX_HIP(launch_seed_apply(p, f0, nf, a->sources, st));
      }
    }
    DLX_HIP(run_adjoint(p, c, f0, nf, a->sources, st));
  }
  Stage sg(p, st, DLX_STAGE_GRAD, p->n_psf);
  DLX_HIP(launch_grad_reduce(p, a->zernike_basis, a->map_basis, a->grad_zernike, a->grad_map, a->grad_sources, a->loss,
                             p->n_chunks, a->grad_intrapixel, st));
  return DLX_OK;
}

dlx_status dlx_graph_capture(dlx_plan* p, const dlx_eval_args* a) {
  if (!p || !a) return DLX_ERR_INVALID_ARG;
  if (!p->cap_stream) DLX_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  if (p->graph_exec) {
    (void)hipGraphExecDestroy(p->graph_exec);
    p->graph_exec = nullptr;
  }
  if (p->graph) {
    (void)hipGraphDestroy(p->graph);
    p->graph = nullptr;
  }
  // No timing-event records inside the graph.
  std::vector<bool> prof{p->profiling};
  p->profiling = false;
  for (dlx_plan* sub : p->subs) {
    prof.push_back(sub->profiling);
    sub->profiling = false;
  }
  DLX_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  const dlx_status s = dlx_eval(p, a, p->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
  p->profiling = prof[0];
  for (size_t k = 0; k < p->subs.size(); ++k) p->subs[k]->profiling = prof[k + 1];
  if (s != DLX_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess || !g) return DLX_ERR_HIP;
  p->graph = g;
  DLX_HIP(hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0));
  return DLX_OK;
}

dlx_status dlx_graph_launch(dlx_plan* p, void* stream) {
  if (!p || !p->graph_exec) return DLX_ERR_INVALID_ARG;
  p->fields_valid = false;   // the replay overwrites the workspace
  for (dlx_plan* sub : p->subs) sub->fields_valid = false;
  DLX_HIP(hipGraphLaunch(p->graph_exec, reinterpret_cast<hipStream_t>(stream)));
  return DLX_OK;
}

}  // extern "C"
