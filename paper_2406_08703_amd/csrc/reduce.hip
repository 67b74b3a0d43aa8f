// HBM-bound stages around the MFT: group reduction of binned partials and
// the pixel response (Section 3), the Poisson / chi-squared loss with the
// pixel-response prior and its gradients (Section 4), and the projections of
// dL/dOPD onto the Zernike basis and the bicubic map. Every reduction runs in
// FP64 in a fixed order, so results are bitwise reproducible.
#include <algorithm>

#include "dlx_internal.h"

namespace dlx {
namespace {

// Intensity, intra-pixel weighting, binning and pixel response (Section 3)
// from the stored focal fields E of frames [f0, f0 + nf):
//   bs[f][s][p] = sum_l w_l sum_{a,b<Q} K[a][b] |E_{f,s,l}[Qp_r + a][Qp_c + b]|^2   (per source, no flux)
//   binned[f][p] = sum_s phi_s bs[f][s][p],  model[f][p] = flat[p] * binned[f][p]
// (binned and model may each be null: the adjoint only needs bs). Block (64,
// kLanes): 64 detector pixels x kLanes rows; wavelength lane k sums
// wavelengths k, k + kLanes, ... and the lanes are added in a fixed order
// (deterministic), the rows taking the (star, lane) items of several stars at
// once (bin_stars). QT > 0 fixes Q at compile time (vector loads along the
// pixel's rows).
constexpr int kLanes = 8;

// element stride of the intra-pixel kernel between detector pixels: 0 (one kernel) or Q^2 (one per pixel)
long long kstride(const dlx_plan* p) { return p->k_per_pixel ? (long long)p->Q * p->Q : 0; }

// Stored column of focal-plane column c: the fields E and seed weights G of a folded plan keep
// columns c < h in place and move c >= h to c + s (s = 0: natural order).
__device__ __forceinline__ int fcol(int c, int h, int s) { return c < h ? c : c + s; }

// |E|^2 of one focal sample at Q = 1, with the rounding fixed (one fused multiply-add) so that the
// one-pixel and four-pixel binning kernels agree bit for bit.
__device__ __forceinline__ float q1_power(float er, float ei) { return __fmaf_rn(er, er, ei * ei); }

// sum over a detector pixel's Q x Q focal samples of K |E|^2 for one PSF: e points at the pixel's
// first focal row; its Q columns start at stored column cb, or (split) straddle the fold's split
// and are mapped one by one from c0.
template <int QT>
__device__ __forceinline__ float pixel_power(const float* e, long long plane, int ld, int Q, int c0, int cb, bool split,
                                             int fh, int fs, const float* kp) {
  float part = 0.f;
  if (split) {   // rare (one pixel column): kept rolled so it costs the common path no registers
#pragma unroll 1
    for (int a = 0; a < Q; ++a)
#pragma unroll 1
      for (int b = 0; b < Q; ++b) {
        const int c = fcol(c0 + b, fh, fs);
        const float er = e[(long long)a * ld + c], ei = e[plane + (long long)a * ld + c];
        float v = er * er + ei * ei;
        if (kp) v *= kp[a * Q + b];
        part += v;
      }
  } else if constexpr (QT == 1) {
    const float er = e[cb], ei = e[plane + cb];
    part = q1_power(er, ei);
    if (kp) part *= kp[0];
  } else if constexpr (QT >= 2) {
    // every load of the pixel (and its kernel weights) is issued before any arithmetic, so that
    // they are in flight together; the weights' branch would otherwise wait for each row in turn
    e += cb;
    float er[QT][QT], ei[QT][QT], kw[QT * QT];
    if constexpr (QT == 3) {   // three columns: not 8- or 16-byte aligned
#pragma unroll
      for (int a = 0; a < QT; ++a)
#pragma unroll
        for (int b = 0; b < QT; ++b) {
          er[a][b] = e[(long long)a * ld + b];
          ei[a][b] = e[plane + (long long)a * ld + b];
        }
    } else {
      typedef float vq __attribute__((ext_vector_type(QT)));
#pragma unroll
      for (int a = 0; a < QT; ++a) {
        const vq vr = *reinterpret_cast<const vq*>(e + (long long)a * ld);
        const vq vi = *reinterpret_cast<const vq*>(e + plane + (long long)a * ld);
#pragma unroll
        for (int b = 0; b < QT; ++b) {
          er[a][b] = vr[b];
          ei[a][b] = vi[b];
        }
      }
    }
    if (kp) {
#pragma unroll
      for (int i = 0; i < QT * QT; ++i) kw[i] = kp[i];
    }
#pragma unroll
    for (int a = 0; a < QT; ++a)
#pragma unroll
      for (int b = 0; b < QT; ++b) {
        float v = er[a][b] * er[a][b] + ei[a][b] * ei[a][b];
        if (kp) v *= kw[a * QT + b];
        part += v;
      }
  } else {
    e += cb;
    for (int a = 0; a < Q; ++a)
      for (int b = 0; b < Q; ++b) {
        const float er = e[(long long)a * ld + b], ei = e[plane + (long long)a * ld + b];
        float v = er * er + ei * ei;
        if (kp) v *= kp[a * Q + b];
        part += v;
      }
  }
  return part;
}

// Per-star binned values of one pixel p of one frame: for every star s,
//   v_s = sum over the kLanes lanes k (in order) of acc_{s,k} = sum_{l = k, k + kLanes, ...} w_l P_{s,l}
// (l in order, P the pixel power above), stored to bs_frame[s npix + p]; returns sum_s phi_s v_s
// (in star order) on the block's first row. The (star, lane) items of up to kItems / min(L, kLanes)
// stars are spread over the block's kLanes rows at once, so that with few wavelengths every row
// still loads (lanes k >= L would only add zeros); the sums do not depend on the grouping.
constexpr int kItems = 64;

template <int QT>
__device__ __forceinline__ double bin_stars(double (*sh)[64], const float* E, long long plane, long long by_psf,
                                            int ld, long long psf0, int S, int L, int Q, int pr, int c0, int cb,
                                            bool split, int fh, int fs, const float* kp, const WlInfo* wl,
                                            const float* src, bool live, float* bs_frame, long long npix,
                                            long long p) {
  const int x = threadIdx.x, y = threadIdx.y;
  const int kl = L < kLanes ? L : kLanes;
  const int sg = kItems / kl;
  double total = 0.0;
  for (int s0 = 0; s0 < S; s0 += sg) {
    const int ns = S - s0 < sg ? S - s0 : sg;
    if (L <= kLanes) {   // one wavelength per item: unrolled so that several items' loads are in flight
#pragma unroll 4
      for (int j = y; j < ns * kl; j += kLanes) {
        const int sl = j / kl, k = j - sl * kl;
        double acc = 0.0;
        if (live) {
          const float* e = E + (psf0 + (long long)(s0 + sl) * L + k) * by_psf + (long long)(Q * pr) * ld;
          acc = fma((double)wl[k].w, (double)pixel_power<QT>(e, plane, ld, Q, c0, cb, split, fh, fs, kp), acc);
        }
        sh[j][x] = acc;
      }
    } else {   // kl == kLanes: the item's star and lane are j / kLanes and j % kLanes
      for (int j = y; j < ns * kLanes; j += kLanes) {
        const int sl = j / kLanes, k = j % kLanes;
        double acc = 0.0;
        if (live)
          for (int l = k; l < L; l += kLanes) {
            const float* e = E + (psf0 + (long long)(s0 + sl) * L + l) * by_psf + (long long)(Q * pr) * ld;
            acc = fma((double)wl[l].w, (double)pixel_power<QT>(e, plane, ld, Q, c0, cb, split, fh, fs, kp), acc);
          }
        sh[j][x] = acc;
      }
    }
    __syncthreads();
    if (ns == 1) {   // one star in the pass (ns is the same for the whole block)
      if (y == 0) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < kLanes; ++k)
          if (k < kl) v += sh[k][x];
        if (live) bs_frame[(long long)s0 * npix + p] = (float)v;
        total = fma((double)src[(long long)s0 * 3 + 2], v, total);
      }
    } else {
      for (int sl = y; sl < ns; sl += kLanes) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < kLanes; ++k)
          if (k < kl) v += sh[sl * kl + k][x];
        if (live) bs_frame[(long long)(s0 + sl) * npix + p] = (float)v;
        sh[sl * kl][x] = v;   // only this thread reads the star's items
      }
      __syncthreads();
      if (y == 0)
        for (int sl = 0; sl < ns; ++sl) total = fma((double)src[(long long)(s0 + sl) * 3 + 2], sh[sl * kl][x], total);
    }
    __syncthreads();
  }
  return total;
}

template <int QT>
__global__ void intensity_kernel(const float* E, long long plane, long long by_psf, int ld, int f0, int F, int S, int L,
                                 int Qr, int Nd, const float* sources, const WlInfo* wl, const float* intrapixel,
                                 long long kst, int fh, int fs, const float* flat, float* bs, float* binned,
                                 float* model) {
  __shared__ double sh[kItems][64];
  const int Q = QT > 0 ? QT : Qr;
  const long long npix = (long long)Nd * Nd;
  const long long p = (long long)blockIdx.x * 64 + threadIdx.x;
  const int f = f0 + blockIdx.y;
  const int y = threadIdx.y;
  const bool live = p < npix && f < F;
  const int pr = live ? (int)(p / Nd) : 0, pc = live ? (int)(p - (long long)pr * Nd) : 0;
  // the intra-pixel kernel of this pixel: shared (kst = 0) or one per pixel (kst = Q^2)
  const float* kp = intrapixel ? intrapixel + (live ? p : 0) * kst : nullptr;
  // this pixel's Q columns: contiguous from cb unless they straddle the fold's split
  const int c0 = Q * pc;
  const bool split = fs != 0 && c0 < fh && c0 + Q > fh;
  const int cb = fcol(c0, fh, fs);
  const double total = bin_stars<QT>(sh, E, plane, by_psf, ld, (long long)(f - f0) * S * L, S, L, Q, pr, c0, cb,
                                     split, fh, fs, kp, wl, sources + (long long)(f < F ? f : 0) * S * 3, live,
                                     bs + (long long)(f - f0) * S * npix, npix, p);
  if (y == 0 && live) {
    const float bv = (float)total;
    if (binned) binned[(long long)f * npix + p] = bv;
    if (model) model[(long long)f * npix + p] = flat[p] * bv;
  }
}

// intensity_kernel at Q = 1 with four adjacent pixels per thread and 16-byte loads (a block covers
// 256 pixels). Launched when N_det and, for a folded plan, the fold's split h are multiples of 4, so
// that the four pixels of a thread share a row and sit contiguous and 16-byte aligned in the stored
// row. Per pixel the arithmetic and the order of every sum are those of intensity_kernel<1>.
constexpr int kItemsV = 16;

__global__ __launch_bounds__(64 * kLanes) void intensity_q1v_kernel(
    const float* E, long long plane, long long by_psf, int ld, int f0, int F, int S, int L, int Nd,
    const float* sources, const WlInfo* wl, const float* intrapixel, long long kst, int fh, int fs,
    const float* flat, float* bs, float* binned, float* model) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  __shared__ double sh[kItemsV][4][64];
  const long long npix = (long long)Nd * Nd;
  const int x = threadIdx.x, y = threadIdx.y;
  const long long p = ((long long)blockIdx.x * 64 + x) * 4;   // first of the thread's four pixels
  const int f = f0 + blockIdx.y;
  const bool live = p < npix && f < F;
  const int pr = live ? (int)(p / Nd) : 0, pc = live ? (int)(p - (long long)pr * Nd) : 0;
  const int cb = fcol(pc, fh, fs);
  float kv[4] = {1.f, 1.f, 1.f, 1.f};
  if (intrapixel && live)
#pragma unroll
    for (int i = 0; i < 4; ++i) kv[i] = intrapixel[(p + i) * kst];
  const float* src = sources + (long long)(f < F ? f : 0) * S * 3;
  float* bsf = bs + (long long)(f - f0) * S * npix;
  const long long psf0 = (long long)(f - f0) * S * L;
  const int kl = L < kLanes ? L : kLanes;
  const int sg = kItemsV / kl > 0 ? kItemsV / kl : 1;
  double total[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s0 = 0; s0 < S; s0 += sg) {
    const int ns = S - s0 < sg ? S - s0 : sg;
    for (int j = y; j < ns * kl; j += kLanes) {
      const int sl = j / kl, k = j - sl * kl;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (live)
        for (int l = k; l < L; l += kLanes) {
          const float* e = E + (psf0 + (long long)(s0 + sl) * L + l) * by_psf + (long long)pr * ld + cb;
          const f4v vr = *reinterpret_cast<const f4v*>(e);
          const f4v vi = *reinterpret_cast<const f4v*>(e + plane);
          const double w = (double)wl[l].w;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float part = q1_power(vr[i], vi[i]);
            if (intrapixel) part *= kv[i];
            acc[i] = fma(w, (double)part, acc[i]);
          }
        }
#pragma unroll
      for (int i = 0; i < 4; ++i) sh[j][i][x] = acc[i];
    }
    __syncthreads();
    for (int sl = y; sl < ns; sl += kLanes) {
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < kl; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] += sh[sl * kl + k][i][x];
      if (live) {
        f4v o;
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = (float)v[i];
        *reinterpret_cast<f4v*>(bsf + (long long)(s0 + sl) * npix + p) = o;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) sh[sl * kl][i][x] = v[i];   // only this thread reads the star's items
    }
    __syncthreads();
    if (y == 0)
      for (int sl = 0; sl < ns; ++sl) {
        const double phi = (double)src[(long long)(s0 + sl) * 3 + 2];
#pragma unroll
        for (int i = 0; i < 4; ++i) total[i] = fma(phi, sh[sl * kl][i][x], total[i]);
      }
    __syncthreads();
  }
  if (y == 0 && live) {
    f4v bv;
#pragma unroll
    for (int i = 0; i < 4; ++i) bv[i] = (float)total[i];
    if (binned) *reinterpret_cast<f4v*>(binned + (long long)f * npix + p) = bv;
    if (model) {
      const f4v fl = *reinterpret_cast<const f4v*>(flat + p);
      *reinterpret_cast<f4v*>(model + (long long)f * npix + p) = fl * bv;
    }
  }
}

constexpr int kLossThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  return t;
}


// The fused evaluation's binning and loss in one pass (in place of intensity_kernel followed by
// loss_kernel<true>): a block of 64 x kLanes threads covers 64 detector pixels and every frame of
// the chunk. For each pixel and frame the kLanes wavelength lanes form the per-star binned values
// (as intensity_kernel); the first wave then forms, as loss_kernel<true> does, the model, the loss
// terms, the residual r, the seed weights G = K flat r and, per star, the block's flux partial
// sum of flat r bs at flux[(f S + s) gridDim.x + block]. The flat-field gradient sums over the
// frames in a register; the loss partial of the block goes to blk[block].
template <int QT>
__device__ __forceinline__ void bin_loss_body(int bx, int nbx, const float* E, long long plane, long long by_psf,
                                              int ld, int f0, int nf, int S, int L, int Qr, int Nd,
                                              const float* sources, const WlInfo* wl, const float* intrapixel,
                                              long long kst, int fh, int fs, const float* flat, const float* data,
                                              int kind, double mu, double inv_s2, float* bs, float* binned,
                                              float* model, float* r_out, double* grad_flat, int accumulate,
                                              double* blk, int* status, float* G, int ldg, long long g_by_frame,
                                              double* flux) {
  __shared__ double sh[kLanes][64];
  const int Q = QT > 0 ? QT : Qr;
  const long long npix = (long long)Nd * Nd;
  const int x = threadIdx.x, y = threadIdx.y;
  const long long p = (long long)bx * 64 + x;
  const bool live = p < npix;
  const int pr = live ? (int)(p / Nd) : 0, pc = live ? (int)(p - (long long)pr * Nd) : 0;
  const float* kp = intrapixel ? intrapixel + (live ? p : 0) * kst : nullptr;
  const int c0 = Q * pc;
  const bool split = fs != 0 && c0 < fh && c0 + Q > fh;
  const int cb = fcol(c0, fh, fs);
  const float fp = live ? flat[p] : 0.f;
  double gf = 0.0, lsum = 0.0;
  int flags = 0;
  for (int fl = 0; fl < nf; ++fl) {
    const int f = f0 + fl;
    // one star per pass (one-frame chunks run with eight or more wavelengths in practice, where
    // bin_stars' grouping gains nothing); the arithmetic and the order of the sums are bin_stars'
    double total = 0.0;
    for (int s = 0; s < S; ++s) {
      double acc = 0.0;
      if (live) {
        for (int l = y; l < L; l += kLanes) {
          const float* e = E + (((long long)fl * S + s) * L + l) * by_psf + (long long)(Q * pr) * ld;
          acc = fma((double)wl[l].w, (double)pixel_power<QT>(e, plane, ld, Q, c0, cb, split, fh, fs, kp), acc);
        }
      }
      sh[y][x] = acc;
      __syncthreads();
      if (y == 0) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < kLanes; ++k)
          if (k < L) v += sh[k][x];
        if (live) bs[((long long)fl * S + s) * npix + p] = (float)v;
        total = fma((double)sources[((long long)f * S + s) * 3 + 2], v, total);
      }
      __syncthreads();
    }
    float h = 0.f;
    if (y == 0 && live) {
      const float bv = (float)total;
      const float mv = fp * bv;
      const long long q = (long long)f * npix + p;
      binned[q] = bv;
      model[q] = mv;
      double m = mv;
      const double d = data[q];
      const double b = bv;
      if (!isfinite(m) || !isfinite(d)) flags |= 1;
      double ell, r;
      if (kind == DLX_LOSS_POISSON) {
        if (m <= 0.0) {
          if (d > 0.0) flags |= 2;
          m = 1e-30;
        }
        ell = m - (d != 0.0 ? d * log(m) : 0.0);
        r = 1.0 - d / m;
      } else {
        const double w = d > 1.0 ? d : 1.0;
        const double dm = m - d;
        ell = 0.5 * dm * dm / w;
        r = dm / w;
      }
      lsum += ell;
      const float rf = (float)r;
      r_out[q] = rf;
      gf += r * b;
      h = fp * rf;
      float* g = G + fl * g_by_frame + (long long)(Q * pr) * ldg;
      for (int a = 0; a < Q; ++a)
        for (int bb = 0; bb < Q; ++bb)
          g[(long long)a * ldg + fcol(Q * pc + bb, fh, fs)] = intrapixel ? h * intrapixel[p * kst + a * Q + bb] : h;
    }
    if (y == 0) {   // the first wave: this frame's flux partials of the block, per star
      for (int s = 0; s < S; ++s) {
        double v = live ? (double)h * (double)bs[((long long)fl * S + s) * npix + p] : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (x == 0) flux[((long long)f * S + s) * nbx + bx] = v;
      }
    }
  }
  if (y == 0) {
    if (live) {
      if (accumulate) {
        grad_flat[p] += gf;
      } else {
        const double dfl = (double)fp - mu;
        lsum += 0.5 * dfl * dfl * inv_s2;
        grad_flat[p] = gf + dfl * inv_s2;
      }
    }
    if (flags) atomicOr(status, flags);  // bit 0: non-finite, bit 1: domain
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
    if (x == 0) blk[bx] = lsum;
  }
}

template <int QT>
__global__ void bin_loss_kernel(const float* E, long long plane, long long by_psf, int ld, int f0, int nf, int S, int L,
                                int Qr, int Nd, const float* sources, const WlInfo* wl, const float* intrapixel,
                                long long kst, int fh, int fs, const float* flat, const float* data, int kind,
                                double mu, double inv_s2, float* bs, float* binned, float* model, float* r_out,
                                double* grad_flat, int accumulate, double* blk, int* status, float* G, int ldg,
                                long long g_by_frame, double* flux) {
  bin_loss_body<QT>(blockIdx.x, gridDim.x, E, plane, by_psf, ld, f0, nf, S, L, Qr, Nd, sources, wl, intrapixel, kst,
                    fh, fs, flat, data, kind, mu, inv_s2, bs, binned, model, r_out, grad_flat, accumulate, blk, status,
                    G, ldg, g_by_frame, flux);
}

// bin_loss_kernel over the one-frame problems of a multi-problem plan in one launch (block table
// entries: problem, pixel block); each problem's arrays at its offsets in the call's packed arrays.
template <int QT>
__global__ void bin_loss_group_kernel(const BinLossArgs* __restrict__ args, const GroupBlock* __restrict__ tab,
                                      GroupCall call) {
  const GroupBlock e = tab[blockIdx.x];
  const BinLossArgs& a = args[e.k];
  const long long im = a.o_img;
  bin_loss_body<QT>(e.x, a.nb, a.E, a.plane, a.by_psf, a.ld, 0, 1, a.S, a.L, a.Q, a.Nd, call.sources + a.o_src, a.wl,
                    call.intrapixel ? call.intrapixel + a.o_k : nullptr, a.kst, a.fh, a.fs, call.flat + a.o_flat,
                    call.data + im, call.kind, call.mu, call.inv_s2, a.bs, call.binned + im, call.model + im,
                    call.r + im, call.grad_flat + a.o_flat, 0, a.blk, a.status, a.G, a.ldg, a.g_by_frame, a.flux);
}

// Outputs of the adjoint seed, when the loss kernel also forms it (fused
// evaluation): seed weights G and flux partials, as seed_weight_kernel below.
struct SeedOut {
  const float* intrapixel;
  long long kst;          // 0: one kernel for all pixels, Q^2: one per pixel
  const float* bs;        // per-source binned [nf][S][npix]
  int Q, Nd, S, ldg;
  int fh, fs;             // stored columns of G (see fcol)
  long long g_by_frame;
  float* G;               // [nf][No][ldg]
  double* flux;           // [F][S][gridDim.x]
};

// Per pixel p: loop over frames f0 <= f < f1, l = m - d ln m (or
// (m-d)^2/(2 max(d,1))), r = dl/dm, and grad_flat[p] = sum_f r B + (F - mu)/sigma^2.
// With `accumulate` the frame sum is added to grad_flat and the prior is left
// out (it was counted by the first frame range); block partials of L go to blk.
// SEED: per frame also G = K flat r (from the stored float r) and the flux
// partials sum_p flat r bs_s of this block.
template <bool SEED>
__global__ void loss_kernel(const float* model, const float* binned, const float* data, const float* flat, int f0,
                            int f1, long long npix, int kind, double mu, double inv_s2, float* r_out,
                            double* grad_flat, int accumulate, double* blk, int* status, SeedOut so) {
  __shared__ double sh[kLossThreads / 64];
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = p < npix;
  const float fp = live ? flat[p] : 0.f;
  double lsum = 0.0, gf = 0.0;
  int flags = 0;
  for (int f = f0; f < f1; ++f) {
    float rf = 0.f;
    if (live) {
      const long long q = (long long)f * npix + p;
      double m = model[q];
      const double d = data[q];
      const double b = binned[q];
      if (!isfinite(m) || !isfinite(d)) flags |= 1;
      double ell, r;
      if (kind == DLX_LOSS_POISSON) {
        if (m <= 0.0) {
          if (d > 0.0) flags |= 2;
          m = 1e-30;
        }
        ell = m - (d != 0.0 ? d * log(m) : 0.0);
        r = 1.0 - d / m;
      } else {
        const double w = d > 1.0 ? d : 1.0;
        const double dm = m - d;
        ell = 0.5 * dm * dm / w;
        r = dm / w;
      }
      lsum += ell;
      rf = (float)r;
      r_out[q] = rf;
      gf += r * b;
    }
    if constexpr (SEED) {
      const int fl = f - f0;
      const float h = fp * rf;
      if (live) {
        const int pr = (int)(p / so.Nd), pc = (int)(p - (long long)pr * so.Nd);
        float* g = so.G + fl * so.g_by_frame + (long long)(so.Q * pr) * so.ldg;
        for (int a = 0; a < so.Q; ++a)
          for (int b = 0; b < so.Q; ++b)
            g[(long long)a * so.ldg + fcol(so.Q * pc + b, so.fh, so.fs)] =
                so.intrapixel ? h * so.intrapixel[p * so.kst + a * so.Q + b] : h;
      }
      for (int s = 0; s < so.S; ++s) {
        const double v = live ? (double)h * (double)so.bs[((long long)fl * so.S + s) * npix + p] : 0.0;
        const double t = block_sum(v, sh);
        if (threadIdx.x == 0) so.flux[((long long)f * so.S + s) * gridDim.x + blockIdx.x] = t;
      }
    }
  }
  if (live) {
    if (accumulate) {
      grad_flat[p] += gf;
    } else {
      const double dfl = (double)fp - mu;
      lsum += 0.5 * dfl * dfl * inv_s2;
      grad_flat[p] = gf + dfl * inv_s2;
    }
  }
  if (flags) atomicOr(status, flags);  // bit 0: non-finite, bit 1: domain
  const double t = block_sum(lsum, sh);
  if (threadIdx.x == 0) blk[blockIdx.x] = t;
}

// L = sum of block partials, one block, fixed order.
__global__ void final_sum_kernel(const double* blk, int n, double* out) {
  __shared__ double sh[1024 / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += blk[i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = t;
}

constexpr int kSeedThreads = 256;

// Seed weights of the adjoint (Section 4) for frames [f0, f0 + nf): per
// detector pixel p = (pr, pc) and focal sample (Q pr + a, Q pc + b),
//   G[f][Q pr + a][Q pc + b] = K[a][b] flat[p] r_f[p]
// (the B3 loader forms Y = w_l phi_s G E from it), and the flux gradient
// partials sum_p flat[p] r_f[p] bs[f][s][p] = sum_l w_l sum G |E_{f,s,l}|^2 per
// (frame, source) and pixel block, at flux[(f S + s) nblk + block].
__global__ void seed_weight_kernel(const float* resid, const float* flat, const float* intrapixel, long long kst,
                                   const float* bs, int f0, int Q, int Nd, int S, int ldg, int fh, int fs,
                                   long long g_by_frame, float* G, int nblk, double* flux) {
  __shared__ double sh[kSeedThreads / 64];
  const long long npix = (long long)Nd * Nd;
  const long long p = (long long)blockIdx.x * kSeedThreads + threadIdx.x;
  const int fl = blockIdx.y;   // frame within the chunk
  const int f = f0 + fl;
  float h = 0.f;
  if (p < npix) {
    const int pr = (int)(p / Nd), pc = (int)(p - (long long)pr * Nd);
    h = flat[p] * resid[(long long)f * npix + p];
    float* g = G + fl * g_by_frame + (long long)(Q * pr) * ldg;
    for (int a = 0; a < Q; ++a)
      for (int b = 0; b < Q; ++b)
        g[(long long)a * ldg + fcol(Q * pc + b, fh, fs)] = intrapixel ? h * intrapixel[p * kst + a * Q + b] : h;
  }
  for (int s = 0; s < S; ++s) {
    double v = 0.0;
    if (p < npix) v = (double)h * (double)bs[((long long)fl * S + s) * npix + p];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kSeedThreads / 64; ++w) t += sh[w];
      flux[((long long)f * S + s) * nblk + blockIdx.x] = t;
    }
    __syncthreads();
  }
}

// Y = (w_l phi_s G_f) E in place for the chunk's PSFs: the separate seed pass,
// used instead of the B3 loader when a frame's seed weights are too large to
// stay cached while B3 streams them. Same arithmetic as the loader.
__global__ void seed_apply_kernel(float* E, long long plane, long long by_psf, const float* G, long long g_by_frame,
                                  long long n4, int blocks_per_psf, int psf0, int f0, int S, int L,
                                  const float* sources, const WlInfo* wl) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const int lb = blockIdx.x / blocks_per_psf;
  const int bx = blockIdx.x - lb * blocks_per_psf;
  const int gb = psf0 + lb;
  const int fs = gb / L;
  const float wphi = wl[gb % L].w * sources[fs * 3 + 2];
  const f4* g = reinterpret_cast<const f4*>(G + (long long)(fs / S - f0) * g_by_frame);
  f4* er = reinterpret_cast<f4*>(E + (long long)lb * by_psf);
  f4* ei = reinterpret_cast<f4*>(E + plane + (long long)lb * by_psf);
  for (long long i = (long long)bx * blockDim.x + threadIdx.x; i < n4; i += (long long)blocks_per_psf * blockDim.x) {
    const f4 sw = wphi * g[i];
    er[i] = sw * er[i];
    ei[i] = sw * ei[i];
  }
}

// Integer-dither mode (Section 3): frame f's images are the N_det x N_det
// window of the enlarged binned plane Bbig [Nb][Nb] at corner win[f]:
//   binned[f][p] = Bbig[win_r + p_r][win_c + p_c],  model[f][p] = flat[p] binned[f][p].
__global__ void window_kernel(const float* Bbig, int Nb, const int* win, int Nd, const float* flat, float* binned,
                              float* model) {
  const long long npix = (long long)Nd * Nd;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (p >= npix) return;
  const int pr = (int)(p / Nd), pc = (int)(p - (long long)pr * Nd);
  const float b = Bbig[(long long)(win[2 * f] + pr) * Nb + win[2 * f + 1] + pc];
  binned[(long long)f * npix + p] = b;
  model[(long long)f * npix + p] = flat[p] * b;
}

// Seed weights of the enlarged plane (integer-dither mode): the adjoint of the
// windows gathers, for enlarged pixel q, h[q] = sum over the frames whose window
// holds q (p = q - win_f) of flat[p] r_f[p], in frame order; then
//   G[Q q_r + a][Q q_c + b] = K[a][b] h[q]
// and the flux partials sum_q h[q] bs_s[q] of this block (one enlarged frame),
// at flux[s nblk + block].
__global__ void seed_gather_kernel(const float* resid, const float* flat, const float* intrapixel, const float* bs,
                                   const int* win, int F, int Nd, int Nb, int Q, int S, int ldg, int fh, int fs,
                                   float* G, double* flux) {
  __shared__ double sh[kSeedThreads / 64];
  const long long nb2 = (long long)Nb * Nb, npix = (long long)Nd * Nd;
  const long long q = (long long)blockIdx.x * kSeedThreads + threadIdx.x;
  float h = 0.f;
  if (q < nb2) {
    const int qr = (int)(q / Nb), qc = (int)(q - (long long)qr * Nb);
    for (int f = 0; f < F; ++f) {
      const int pr = qr - win[2 * f], pc = qc - win[2 * f + 1];
      if (pr >= 0 && pr < Nd && pc >= 0 && pc < Nd) {
        const long long p = (long long)pr * Nd + pc;
        h += flat[p] * resid[(long long)f * npix + p];
      }
    }
    float* g = G + (long long)(Q * qr) * ldg;
    for (int a = 0; a < Q; ++a)
      for (int b = 0; b < Q; ++b)
        g[(long long)a * ldg + fcol(Q * qc + b, fh, fs)] = intrapixel ? h * intrapixel[a * Q + b] : h;
  }
  for (int s = 0; s < S; ++s) {
    double v = q < nb2 ? (double)h * (double)bs[(long long)s * nb2 + q] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kSeedThreads / 64; ++w) t += sh[w];
      flux[(long long)s * gridDim.x + blockIdx.x] = t;
    }
    __syncthreads();
  }
}

// Partials of dL/dK, the gradient with respect to the intra-pixel kernel (it
// enters the binning linearly): per detector pixel p of frame f (one thread),
//   h = flat[p] r_f[p]   (integer-dither mode: the window gather of the
//                         enlarged plane, as in seed_gather_kernel)
//   v[a][b] = h sum_s sum_l w_l phi_s |E_{f,s,l}[Q p_r + a][Q p_c + b]|^2,
// summed over the block's pixels into part[(f nblk + block) Q^2 + a Q + b].
// With one kernel per pixel (gpix non-null) the pixel sum is dropped: the block runs every frame
// of the chunk (grid.y = 1) and writes gpix[p][a][b], or adds to it for a chunk after the first.
template <int QT>
__global__ __launch_bounds__(kSeedThreads) void kgrad_kernel(const float* E, long long plane, long long by_psf, int ld, int f0, int S, int L,
                             int Nd, const float* sources, const WlInfo* wl, const float* flat, const float* resid,
                             const int* win, int F_img, int Nd_img, int fh, int fs, double* part, double* gpix,
                             int nf_pix, int accumulate) {
  constexpr int Q2 = QT * QT;
  __shared__ double sh[Q2][kSeedThreads / 64];
  const long long npix = (long long)Nd * Nd;
  const long long p = (long long)blockIdx.x * kSeedThreads + threadIdx.x;
  double acc[Q2];
#pragma unroll
  for (int k = 0; k < Q2; ++k) acc[k] = 0.0;
  // frames of this block: one (blockIdx.y) for the shared kernel, all nf_pix of the chunk per pixel
  const int fl0 = gpix ? 0 : blockIdx.y, fl1 = gpix ? nf_pix : blockIdx.y + 1;
  for (int fl = fl0; fl < fl1; ++fl) {
    const int f = f0 + fl;
    if (p < npix) {
      const int pr = (int)(p / Nd), pc = (int)(p - (long long)pr * Nd);
      float h = 0.f;
      if (win) {
        const long long nimg = (long long)Nd_img * Nd_img;
        for (int g = 0; g < F_img; ++g) {
          const int ir = pr - win[2 * g], ic = pc - win[2 * g + 1];
          if (ir >= 0 && ir < Nd_img && ic >= 0 && ic < Nd_img) {
            const long long q = (long long)ir * Nd_img + ic;
            h += flat[q] * resid[(long long)g * nimg + q];
          }
        }
      } else {
        h = flat[p] * resid[(long long)f * npix + p];
      }
      double v[Q2];
#pragma unroll
      for (int k = 0; k < Q2; ++k) v[k] = 0.0;
      for (int s = 0; s < S; ++s) {
        const float phi = sources[((long long)f * S + s) * 3 + 2];
        for (int l = 0; l < L; ++l) {
          const float* e = E + (((long long)fl * S + s) * L + l) * by_psf + (long long)(QT * pr) * ld;
          const float wphi = wl[l].w * phi;
#pragma unroll
          for (int a = 0; a < QT; ++a)
#pragma unroll
            for (int b = 0; b < QT; ++b) {
              const int c = fcol(QT * pc + b, fh, fs);
              const float er = e[(long long)a * ld + c], ei = e[plane + (long long)a * ld + c];
              v[a * QT + b] += (double)(wphi * (er * er + ei * ei));
            }
        }
      }
#pragma unroll
      for (int k = 0; k < Q2; ++k) acc[k] += v[k] * (double)h;
    }
  }
  if (gpix) {
    if (p < npix) {
#pragma unroll
      for (int k = 0; k < Q2; ++k) gpix[p * Q2 + k] = (accumulate ? gpix[p * Q2 + k] : 0.0) + acc[k];
    }
    return;
  }
  const int f = f0 + blockIdx.y;
#pragma unroll
  for (int k = 0; k < Q2; ++k) {
    double v = acc[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < Q2) {
    double t = 0.0;
    for (int w = 0; w < kSeedThreads / 64; ++w) t += sh[threadIdx.x][w];
    part[((long long)f * gridDim.x + blockIdx.x) * Q2 + threadIdx.x] = t;
  }
}

// gopd[p] = sum_g gpart[g][p]
__device__ __forceinline__ void gopd_body(int bx, const float* gpart, int G, long long npix, double* gopd) {
  const long long p = (long long)bx * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  double acc = 0.0;
#pragma unroll 8
  for (int g = 0; g < G; ++g) acc += (double)gpart[(long long)g * npix + p];
  gopd[p] = acc;
}

__global__ void gopd_reduce_kernel(const float* gpart, int G, long long npix, double* gopd) {
  gopd_body(blockIdx.x, gpart, G, npix, gopd);
}

// Zernike projection dL/dc_j = sum_p Z_j[p] gopd[p], in two deterministic passes:
// block (term group of 8, pixel chunk) writes part[chunk][j]; zproj_final sums chunks.
constexpr int kZGroup = 8;

__device__ __forceinline__ void zproj_body(int bx, int by, const float* Z, const double* gopd, int Nz, long long npix,
                                           long long chunk, double* part) {
  __shared__ double sh[4][kZGroup];
  const int j0 = bx * kZGroup;
  const long long p_begin = (long long)by * chunk;
  const long long p_end = p_begin + chunk < npix ? p_begin + chunk : npix;
  double acc[kZGroup];
#pragma unroll
  for (int q = 0; q < kZGroup; ++q) acc[q] = 0.0;
  // four consecutive pixels per thread and step (chunk is a multiple of 1024)
  for (long long p = p_begin + 4 * threadIdx.x; p < p_end; p += 4 * blockDim.x) {
    const bool full = p + 4 <= p_end && (npix & 3) == 0 && (reinterpret_cast<uintptr_t>(Z) & 15) == 0;
    double g[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) g[e] = (p + e < p_end) ? gopd[p + e] : 0.0;
#pragma unroll
    for (int q = 0; q < kZGroup; ++q) {
      if (j0 + q >= Nz) break;
      const float* z = Z + (long long)(j0 + q) * npix + p;
      if (full) {
        const float4 v = *reinterpret_cast<const float4*>(z);
        acc[q] += (double)v.x * g[0] + (double)v.y * g[1] + (double)v.z * g[2] + (double)v.w * g[3];
      } else {
        for (int e = 0; e < 4; ++e)
          if (p + e < p_end) acc[q] += (double)z[e] * g[e];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kZGroup; ++q) {
    double v = acc[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < kZGroup && j0 + (int)threadIdx.x < Nz) {
    const int q = threadIdx.x;
    part[(long long)by * Nz + j0 + q] = sh[0][q] + sh[1][q] + sh[2][q] + sh[3][q];
  }
}

__global__ void zproj_partial_kernel(const float* Z, const double* gopd, int Nz, long long npix, long long chunk,
                                     double* part) {
  zproj_body(blockIdx.x, blockIdx.y, Z, gopd, Nz, npix, chunk, part);
}

// The bicubic-map gradient B^T gopd B in two products over the pupil index, each output a
// fixed-order FP64 sum: block of kMapWaves waves, lane = output column k (64 at a time), wave w
// sums the terms w, w + kMapWaves, ... and the wave sums are added in wave order.
constexpr int kMapWaves = 16;

// tmp2[m][k] = sum_n gopd[m][n] B[n][k]   (block m)
__global__ __launch_bounds__(64 * kMapWaves) void map_grad1_kernel(const double* gopd, const float* Bm, int Ni, int Nmap, double* tmp2) {
  __shared__ double sh[kMapWaves][64];
  const int m = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* g = gopd + (long long)m * Ni;
  for (int k0 = 0; k0 < Nmap; k0 += 64) {
    const int k = k0 + lane;
    double acc = 0.0;
    if (k < Nmap) {
#pragma unroll 4
      for (int n = w; n < Ni; n += kMapWaves) acc += g[n] * (double)Bm[(long long)n * Nmap + k];
    }
    sh[w][lane] = acc;
    __syncthreads();
    if (w == 0 && k < Nmap) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < kMapWaves; ++i) t += sh[i][lane];
      tmp2[(long long)m * Nmap + k] = t;
    }
    __syncthreads();
  }
}

// grad_C[j][k] = sum_m B[m][j] tmp2[m][k]   (block j)
__global__ __launch_bounds__(64 * kMapWaves) void map_grad2_kernel(const double* tmp2, const float* Bm, int Ni, int Nmap, double* grad) {
  __shared__ double sh[kMapWaves][64];
  const int j = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int k0 = 0; k0 < Nmap; k0 += 64) {
    const int k = k0 + lane;
    double acc = 0.0;
    if (k < Nmap) {
#pragma unroll 4
      for (int m = w; m < Ni; m += kMapWaves)
        acc += (double)Bm[(long long)m * Nmap + j] * tmp2[(long long)m * Nmap + k];
    }
    sh[w][lane] = acc;
    __syncthreads();
    if (w == 0 && k < Nmap) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < kMapWaves; ++i) t += sh[i][lane];
      grad[(long long)j * Nmap + k] = t;
    }
    __syncthreads();
  }
}

// The last reductions of an evaluation in one launch, 256 threads per block,
// each a fixed-order FP64 sum:
//   blocks [0, Nz):          dL/dc_j = sum over pixel chunks of the projection partials;
//   blocks [Nz, Nz + F S):   grad_sources[f][s] = position partials summed over
//                            wavelengths and tiles, flux partials over pixel blocks;
//   block Nz + F S (if loss): L = sum of the loss block partials;
//   the last Q^2 blocks (if gK): dL/dK[a][b] = sum of the intra-pixel partials.
__device__ __forceinline__ void finalize_body(int b, const double* zpart, int Nz, int nchunks, double* gz,
                                              const double* flux, int seed_blocks, const double* pos, int tiles_b4,
                                              int L, int FS, double* gsrc, const double* lossblk, int nloss,
                                              double* loss, const double* kpart, int nkpart, int Q2, double* gK) {
  __shared__ double sh[3][4];
  const int w = threadIdx.x >> 6;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  if (b < Nz) {
    for (int c = threadIdx.x; c < nchunks; c += 256) v0 += zpart[(long long)c * Nz + b];
  } else if (b < Nz + FS) {
    const int fs = b - Nz;
    const long long b0 = (long long)fs * L;
    for (int i = threadIdx.x; i < L * tiles_b4; i += 256) {
      const long long q = (b0 * tiles_b4 + i) * 2;
      v0 += pos[q];
      v1 += pos[q + 1];
    }
    for (int i = threadIdx.x; i < seed_blocks; i += 256) v2 += flux[(long long)fs * seed_blocks + i];
  } else if (loss && b == Nz + FS) {
    for (int i = threadIdx.x; i < nloss; i += 256) v0 += lossblk[i];
  } else {
    const int k = b - Nz - FS - (loss ? 1 : 0);
    for (int i = threadIdx.x; i < nkpart; i += 256) v0 += kpart[(long long)i * Q2 + k];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v0 += __shfl_xor(v0, o, 64);
    v1 += __shfl_xor(v1, o, 64);
    v2 += __shfl_xor(v2, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = v0;
    sh[1][w] = v1;
    sh[2][w] = v2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    const double t = sh[k][0] + sh[k][1] + sh[k][2] + sh[k][3];
    if (b < Nz) {
      if (k == 0) gz[b] = t;
    } else if (b < Nz + FS) {
      gsrc[(b - Nz) * 3 + k] = t;
    } else if (loss && b == Nz + FS) {
      if (k == 0) loss[0] = t;
    } else if (k == 0) {
      gK[b - Nz - FS - (loss ? 1 : 0)] = t;
    }
  }
}

__global__ void finalize_kernel(const double* zpart, int Nz, int nchunks, double* gz, const double* flux,
                                int seed_blocks, const double* pos, int tiles_b4, int L, int FS, double* gsrc,
                                const double* lossblk, int nloss, double* loss, const double* kpart, int nkpart,
                                int Q2, double* gK) {
  finalize_body(blockIdx.x, zpart, Nz, nchunks, gz, flux, seed_blocks, pos, tiles_b4, L, FS, gsrc, lossblk, nloss,
                loss, kpart, nkpart, Q2, gK);
}

// The last reductions of every problem of a multi-problem plan, each a grouped launch (block
// table entries: problem and the block in that problem's own grid): gopd_reduce_kernel,
// zproj_partial_kernel and finalize_kernel (with the loss, without dL/dK).
__global__ __launch_bounds__(256) void gopd_group_kernel(const GradArgs* __restrict__ args,
                                                         const GroupBlock* __restrict__ tab) {
  const GroupBlock e = tab[blockIdx.x];
  const GradArgs& a = args[e.k];
  gopd_body(e.x, a.gpart, a.G, a.npix, a.gopd);
}

__global__ __launch_bounds__(256) void zproj_group_kernel(const GradArgs* __restrict__ args,
                                                          const GroupBlock* __restrict__ tab, const float* Z) {
  const GroupBlock e = tab[blockIdx.x];
  const GradArgs& a = args[e.k];
  zproj_body(e.x, e.y, Z + a.o_z, a.gopd, a.Nz, a.npix, a.zchunk, a.zpart);
}

__global__ __launch_bounds__(256) void finalize_group_kernel(const GradArgs* __restrict__ args,
                                                             const GroupBlock* __restrict__ tab, GroupCall call) {
  const GroupBlock e = tab[blockIdx.x];
  const GradArgs& a = args[e.k];
  finalize_body(e.x, a.zpart, a.Nz, a.nchunks, a.Nz ? call.grad_zernike + a.o_c : nullptr, a.flux, a.flux_blocks,
                a.pos, a.tiles_b4, a.L, a.FS, call.grad_sources + a.o_src, a.lossblk, a.nloss, call.loss + a.o_loss,
                nullptr, 0, 0, nullptr);
}

}  // namespace

hipError_t launch_intensity(dlx_plan* p, int f0, int nf, const float* sources, const float* intrapixel,
                            const float* flat, float* binned, float* model, hipStream_t st) {
  const long long npix = (long long)p->Nd * p->Nd;
  const dim3 grid((unsigned)((npix + 63) / 64), nf), blk(64, kLanes);
  const long long plane = (long long)p->chunk_psf * p->No * p->ldNo, by = (long long)p->No * p->ldNo;
#define DLX_INTENSITY(QT)                                                                                         \
  hipLaunchKernelGGL(intensity_kernel<QT>, grid, blk, 0, st, p->d_Y, plane, by, p->ldNo, f0, p->F, p->S, p->L, \
                     p->Q, p->Nd, sources, p->d_wl, intrapixel, kstride(p), p->hNo(), p->sNo(), flat, p->d_bs,   \
                     binned, model)
  // the four-pixel kernel moves flat, binned and model in 16-byte vectors: caller pointers must be
  // 16-byte aligned (packed multi-problem arrays are not after a problem with an odd pixel count)
  const bool aligned16 = ((reinterpret_cast<uintptr_t>(flat) | reinterpret_cast<uintptr_t>(binned) |
                           reinterpret_cast<uintptr_t>(model)) & 15) == 0;
  if (p->Q == 1 && p->Nd % 4 == 0 && (!p->fold || p->hNo() % 4 == 0) && aligned16) {
    const dim3 grid4((unsigned)((npix / 4 + 63) / 64), nf);
    hipLaunchKernelGGL(intensity_q1v_kernel, grid4, blk, 0, st, p->d_Y, plane, by, p->ldNo, f0, p->F, p->S, p->L,
                       p->Nd, sources, p->d_wl, intrapixel, kstride(p), p->hNo(), p->sNo(), flat, p->d_bs, binned,
                       model);
    return hipGetLastError();
  }
  switch (p->Q) {
    case 1: DLX_INTENSITY(1); break;
    case 2: DLX_INTENSITY(2); break;
    case 3: DLX_INTENSITY(3); break;
    case 4: DLX_INTENSITY(4); break;
    default: DLX_INTENSITY(0); break;
  }
#undef DLX_INTENSITY
  return hipGetLastError();
}

int seed_block_count(long long npix) { return (int)((npix + kSeedThreads - 1) / kSeedThreads); }

hipError_t launch_seed(dlx_plan* p, int f0, int nf, const float* flat, const float* resid, const float* intrapixel,
                       hipStream_t st) {
  p->flux_blocks = p->seed_blocks;
  hipLaunchKernelGGL(seed_weight_kernel, dim3(p->seed_blocks, nf), dim3(kSeedThreads), 0, st, resid, flat, intrapixel,
                     kstride(p), p->d_bs, f0, p->Q, p->Nd, p->S, p->ldNo, p->hNo(), p->sNo(), (long long)p->No * p->ldNo,
                     p->d_G, p->seed_blocks, p->d_flux);
  return hipGetLastError();
}

hipError_t launch_seed_apply(dlx_plan* p, int f0, int nf, const float* sources, hipStream_t st) {
  const int nc = nf * p->S * p->L;
  const long long n4 = (long long)p->No * p->ldNo / 4;
  const int bpp = (int)std::min<long long>(64, (n4 + 255) / 256);
  hipLaunchKernelGGL(seed_apply_kernel, dim3(nc * bpp), dim3(256), 0, st, p->d_Y,
                     (long long)p->chunk_psf * p->No * p->ldNo, (long long)p->No * p->ldNo, p->d_G,
                     (long long)p->No * p->ldNo, n4, bpp, f0 * p->S * p->L, f0, p->S, p->L, sources, p->d_wl);
  return hipGetLastError();
}

hipError_t launch_window(dlx_plan* p, const float* flat, float* binned, float* model, hipStream_t st) {
  const long long npix = (long long)p->Nd_img * p->Nd_img;
  hipLaunchKernelGGL(window_kernel, dim3((unsigned)((npix + 255) / 256), p->F_img), dim3(256), 0, st, p->d_Bbig,
                     p->Nd, p->d_win, p->Nd_img, flat, binned, model);
  return hipGetLastError();
}

hipError_t launch_seed_gather(dlx_plan* p, const float* flat, const float* resid, const float* intrapixel,
                              hipStream_t st) {
  p->flux_blocks = p->seed_blocks;
  hipLaunchKernelGGL(seed_gather_kernel, dim3(p->seed_blocks), dim3(kSeedThreads), 0, st, resid, flat, intrapixel,
                     p->d_bs, p->d_win, p->F_img, p->Nd_img, p->Nd, p->Q, p->S, p->ldNo, p->hNo(), p->sNo(), p->d_G,
                     p->d_flux);
  return hipGetLastError();
}

// dL/dK partials of frames [f0, f0 + nf) (one enlarged frame in integer-dither mode); Q <= 4.
// gK: the caller's [Nd][Nd][Q][Q] output when the plan has one kernel per pixel (written by the
// first chunk, added to by the others); otherwise ignored and the partials go to d_kpart.
hipError_t launch_kgrad(dlx_plan* p, int f0, int nf, const float* sources, const float* flat, const float* resid,
                        double* gK, hipStream_t st) {
  const long long plane = (long long)p->chunk_psf * p->No * p->ldNo, by = (long long)p->No * p->ldNo;
  const dim3 grid(p->seed_blocks, p->k_per_pixel ? 1 : nf), blk(kSeedThreads);
  const int* win = p->dither ? p->d_win : nullptr;
  double* gpix = p->k_per_pixel ? gK : nullptr;
#define DLX_KGRAD(QT)                                                                                          \
  hipLaunchKernelGGL(kgrad_kernel<QT>, grid, blk, 0, st, p->d_Y, plane, by, p->ldNo, f0, p->S, p->L, p->Nd,  \
                     sources, p->d_wl, flat, resid, win, p->F_img, p->Nd_img, p->hNo(), p->sNo(), p->d_kpart, gpix, \
                     nf, f0 > 0 ? 1 : 0)
  switch (p->Q) {
    case 1: DLX_KGRAD(1); break;
    case 2: DLX_KGRAD(2); break;
    case 3: DLX_KGRAD(3); break;
    case 4: DLX_KGRAD(4); break;
    default: return hipErrorInvalidValue;
  }
#undef DLX_KGRAD
  return hipGetLastError();
}

int loss_block_count(long long npix) { return (int)((npix + kLossThreads - 1) / kLossThreads); }

// Loss terms of frames [f0, f0 + nf); block partials at slot `chunk`. The
// loss itself is summed over the slots by launch_loss_final or the finalize
// kernel. With seed_intrapixel_or_none non-null (pointing at the intra-pixel
// kernel, itself possibly null) the adjoint seed weights and flux partials
// of these frames are formed as well.
hipError_t launch_loss(dlx_plan* p, int f0, int nf, int chunk, const float* model, const float* binned,
                       const float* data, const float* flat, int kind, double mu, double sigma, float* r, double* gflat,
                       const float* const* seed_intrapixel_or_none, hipStream_t st) {
  const long long npix = (long long)p->Nd_img * p->Nd_img;
  const int nb = loss_block_count(npix);
  const double inv_s2 = 1.0 / (sigma * sigma);
  double* blk = p->d_lossblk + (long long)chunk * nb;
  p->lossblk_chunk = nb;
  if (seed_intrapixel_or_none) {
    p->flux_blocks = nb;
    const SeedOut so{*seed_intrapixel_or_none, kstride(p), p->d_bs, p->Q, p->Nd, p->S, p->ldNo, p->hNo(), p->sNo(),
                     (long long)p->No * p->ldNo, p->d_G, p->d_flux};
    hipLaunchKernelGGL(loss_kernel<true>, dim3(nb), dim3(kLossThreads), 0, st, model, binned, data, flat, f0, f0 + nf,
                       npix, kind, mu, inv_s2, r, gflat, chunk > 0 ? 1 : 0, blk, p->d_status, so);
  } else {
    hipLaunchKernelGGL(loss_kernel<false>, dim3(nb), dim3(kLossThreads), 0, st, model, binned, data, flat, f0,
                       f0 + nf, npix, kind, mu, inv_s2, r, gflat, chunk > 0 ? 1 : 0, blk, p->d_status, SeedOut{});
  }
  return hipGetLastError();
}

int bin_loss_block_count(long long npix) { return (int)((npix + 63) / 64); }

// dlx_eval's binning, loss, residual, seed weights and flux partials of frames [f0, f0 + nf) in
// one launch (ordinary frames; the integer-dither mode keeps its windows and gather). One block
// per 64 pixels; its loss partials at slot `chunk`, its flux partials per (frame, star).
hipError_t launch_bin_loss(dlx_plan* p, int f0, int nf, int chunk, const float* sources, const float* intrapixel,
                           const float* flat, const float* data, int kind, double mu, double sigma, float* binned,
                           float* model, float* r, double* gflat, hipStream_t st) {
  const long long npix = (long long)p->Nd * p->Nd;
  const int nb = bin_loss_block_count(npix);
  const double inv_s2 = 1.0 / (sigma * sigma);
  double* blk = p->d_lossblk + (long long)chunk * nb;
  const long long plane = (long long)p->chunk_psf * p->No * p->ldNo, by = (long long)p->No * p->ldNo;
  const dim3 grid(nb), blkdim(64, kLanes);
  p->flux_blocks = nb;
  p->lossblk_chunk = nb;
#define DLX_BIN_LOSS(QT)                                                                                           \
  hipLaunchKernelGGL(bin_loss_kernel<QT>, grid, blkdim, 0, st, p->d_Y, plane, by, p->ldNo, f0, nf, p->S, p->L,  \
                     p->Q, p->Nd, sources, p->d_wl, intrapixel, kstride(p), p->hNo(), p->sNo(), flat, data, kind, \
                     mu, inv_s2, p->d_bs, binned, model, r, gflat, chunk > 0 ? 1 : 0, blk, p->d_status, p->d_G,    \
                     p->ldNo, (long long)p->No * p->ldNo, p->d_flux)
  switch (p->Q) {
    case 1: DLX_BIN_LOSS(1); break;
    case 2: DLX_BIN_LOSS(2); break;
    case 3: DLX_BIN_LOSS(3); break;
    case 4: DLX_BIN_LOSS(4); break;
    default: DLX_BIN_LOSS(0); break;
  }
#undef DLX_BIN_LOSS
  return hipGetLastError();
}

hipError_t launch_bin_loss_group(int qt, const BinLossArgs* args, const GroupBlock* tab, int n_blocks,
                                 const GroupCall& call, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  const dim3 grid(n_blocks), blk(64, kLanes);
  switch (qt) {
    case 1: hipLaunchKernelGGL(bin_loss_group_kernel<1>, grid, blk, 0, st, args, tab, call); break;
    case 2: hipLaunchKernelGGL(bin_loss_group_kernel<2>, grid, blk, 0, st, args, tab, call); break;
    case 3: hipLaunchKernelGGL(bin_loss_group_kernel<3>, grid, blk, 0, st, args, tab, call); break;
    case 4: hipLaunchKernelGGL(bin_loss_group_kernel<4>, grid, blk, 0, st, args, tab, call); break;
    default: hipLaunchKernelGGL(bin_loss_group_kernel<0>, grid, blk, 0, st, args, tab, call); break;
  }
  return hipGetLastError();
}

hipError_t launch_grad_group(const GradArgs* args, const GroupBlock* gopd_tab, int n_gopd, const GroupBlock* z_tab,
                             int n_z, const GroupBlock* fin_tab, int n_fin, const GroupCall& call, hipStream_t st) {
  if (n_gopd > 0) hipLaunchKernelGGL(gopd_group_kernel, dim3(n_gopd), dim3(256), 0, st, args, gopd_tab);
  if (n_z > 0) hipLaunchKernelGGL(zproj_group_kernel, dim3(n_z), dim3(256), 0, st, args, z_tab, call.zbasis);
  if (n_fin > 0) hipLaunchKernelGGL(finalize_group_kernel, dim3(n_fin), dim3(256), 0, st, args, fin_tab, call);
  return hipGetLastError();
}

// dlx_loss_grad's two launches (loss_kernel without the seed, then final_sum_kernel) over
// caller-given buffers: blk holds loss_block_count(npix) doubles, status one int (OR-ed flags).
hipError_t launch_loss_plain(int nf, long long npix, const float* model, const float* binned, const float* data,
                             const float* flat, int kind, double mu, double sigma, float* r, double* gflat,
                             double* blk, int* status, double* loss, hipStream_t st) {
  const int nb = loss_block_count(npix);
  hipLaunchKernelGGL(loss_kernel<false>, dim3(nb), dim3(kLossThreads), 0, st, model, binned, data, flat, 0, nf, npix,
                     kind, mu, 1.0 / (sigma * sigma), r, gflat, 0, blk, status, SeedOut{});
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(1024), 0, st, blk, nb, loss);
  return hipGetLastError();
}

hipError_t launch_loss_final(dlx_plan* p, int n_chunks, double* loss, hipStream_t st) {
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(1024), 0, st, p->d_lossblk, p->lossblk_chunk * n_chunks, loss);
  return hipGetLastError();
}

// pixel chunks of the Zernike projection: about 2048 blocks in all, each
// thread covering at least 8 pixels (latency of the scattered loads hides
// behind each thread's own loop)
int zproj_chunks(long long npix, int Nz) {
  const int groups = (Nz + kZGroup - 1) / kZGroup;
  long long c = 2048 / (groups > 0 ? groups : 1);
  c = c < 1 ? 1 : c;
  const long long maxc = (npix + 1023) / 1024;
  return (int)(c < maxc ? c : maxc);
}

// dL/dOPD, its projections and the source gradients; with `loss` also the
// loss of dlx_eval's n_chunks block-partial slots.
hipError_t launch_grad_reduce(dlx_plan* p, const float* Z, const float* Bm, double* gz, double* gmap, double* gsrc,
                              double* loss, int loss_chunks, double* gK, hipStream_t st) {
  const long long npix = (long long)p->Ni * p->Ni;
  const int G = p->b4_groups_max * p->b4_ksplit;
  hipLaunchKernelGGL(gopd_reduce_kernel, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, p->d_gpart, G, npix,
                     p->d_gopd);
  int nch = 1;
  if (p->Nz > 0) {
    nch = zproj_chunks(npix, p->Nz);
    const long long chunk = ((npix + nch - 1) / nch + 1023) / 1024 * 1024;
    hipLaunchKernelGGL(zproj_partial_kernel, dim3((p->Nz + kZGroup - 1) / kZGroup, nch), dim3(256), 0, st, Z,
                       p->d_gopd, p->Nz, npix, chunk, p->d_zpart);
  }
  if (p->Nmap > 0) {
    hipLaunchKernelGGL(map_grad1_kernel, dim3(p->Ni), dim3(64 * kMapWaves), 0, st, p->d_gopd, Bm, p->Ni, p->Nmap,
                       p->d_tmp2);
    hipLaunchKernelGGL(map_grad2_kernel, dim3(p->Nmap), dim3(64 * kMapWaves), 0, st, p->d_tmp2, Bm, p->Ni, p->Nmap,
                       gmap);
  }
  const int FS = p->F * p->S;
  const int Q2 = p->Q * p->Q;
  // one kernel per pixel: launch_kgrad already wrote gK in full
  if (p->k_per_pixel) gK = nullptr;
  hipLaunchKernelGGL(finalize_kernel, dim3(p->Nz + FS + (loss ? 1 : 0) + (gK ? Q2 : 0)), dim3(256), 0, st,
                     p->d_zpart, p->Nz, nch, gz, p->d_flux, p->flux_blocks, p->d_pos, p->tiles_b4 * p->b4_ksplit, p->L,
                     FS, gsrc, p->d_lossblk, p->lossblk_chunk * loss_chunks, loss, p->d_kpart, p->F * p->seed_blocks, Q2,
                     gK);
  return hipGetLastError();
}

}  // namespace dlx
