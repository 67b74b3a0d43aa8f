// HBM-bound stages around the MFT: group reduction of binned partials and
// the pixel response (Section 3), the Poisson / chi-squared loss with the
// pixel-response prior and its gradients (Section 4), and the projections of
// dL/dOPD onto the Zernike basis and the bicubic map. Every reduction runs in
// FP64 in a fixed order, so results are bitwise reproducible.
#include "dlx_internal.h"

namespace dlx {
namespace {

// Intensity, intra-pixel weighting, binning and pixel response (Section 3)
// from the stored focal fields E of frames [f0, f0 + nf):
//   binned[f][p] = sum_s sum_l w_l phi_s sum_{a,b<Q} K[a][b] |E[Qp_r + a][Qp_c + b]|^2,
//   model[f][p] = flat[p] * binned[f][p].
// Block (64, 4): 64 detector pixels x 4 PSF lanes; lane y sums PSFs
// y, y + 4, ... and the lanes are added in a fixed order (deterministic).
// QT > 0 fixes Q at compile time (vector loads along the pixel's rows).
template <int QT>
__global__ void intensity_kernel(const float* E, long long plane, long long by_psf, int ld, int f0, int F, int S, int L,
                                 int Qr, int Nd, const float* sources, const WlInfo* wl, const float* intrapixel,
                                 const float* flat, float* binned, float* model) {
  __shared__ double sh[4][64];
  const int Q = QT > 0 ? QT : Qr;
  const long long npix = (long long)Nd * Nd;
  const long long p = (long long)blockIdx.x * 64 + threadIdx.x;
  const int f = f0 + blockIdx.y;
  const int y = threadIdx.y;
  double acc = 0.0;
  if (p < npix && f < F) {
    const int pr = (int)(p / Nd), pc = (int)(p - (long long)pr * Nd);
    const int SL = S * L;
    for (int q = y; q < SL; q += 4) {
      const int s = q / L, l = q - s * L;
      const long long lb = (long long)(f - f0) * SL + q;
      const float* e = E + lb * by_psf + (long long)(Q * pr) * ld + Q * pc;
      float part = 0.f;
      if constexpr (QT == 4 || QT == 2) {
        typedef float vq __attribute__((ext_vector_type(QT)));
#pragma unroll
        for (int a = 0; a < QT; ++a) {
          const vq vr = *reinterpret_cast<const vq*>(e + (long long)a * ld);
          const vq vi = *reinterpret_cast<const vq*>(e + plane + (long long)a * ld);
#pragma unroll
          for (int b = 0; b < QT; ++b) {
            float v = vr[b] * vr[b] + vi[b] * vi[b];
            if (intrapixel) v *= intrapixel[a * QT + b];
            part += v;
          }
        }
      } else {
        for (int a = 0; a < Q; ++a)
          for (int b = 0; b < Q; ++b) {
            const float er = e[(long long)a * ld + b], ei = e[plane + (long long)a * ld + b];
            float v = er * er + ei * ei;
            if (intrapixel) v *= intrapixel[a * Q + b];
            part += v;
          }
      }
      acc += (double)(wl[l].w * sources[((long long)f * S + s) * 3 + 2]) * (double)part;
    }
  }
  sh[y][threadIdx.x] = acc;
  __syncthreads();
  if (y == 0 && p < npix && f < F) {
    const float bv = (float)(sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x]);
    binned[(long long)f * npix + p] = bv;
    model[(long long)f * npix + p] = flat[p] * bv;
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

// Per pixel p: loop over frames f0 <= f < f1, l = m - d ln m (or
// (m-d)^2/(2 max(d,1))), r = dl/dm, and grad_flat[p] = sum_f r B + (F - mu)/sigma^2.
// With `accumulate` the frame sum is added to grad_flat and the prior is left
// out (it was counted by the first frame range); block partials of L go to blk.
__global__ void loss_kernel(const float* model, const float* binned, const float* data, const float* flat, int f0,
                            int f1, long long npix, int kind, double mu, double inv_s2, float* r_out,
                            double* grad_flat, int accumulate, double* blk, int* status) {
  __shared__ double sh[kLossThreads / 64];
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double lsum = 0.0;
  int flags = 0;
  if (p < npix) {
    double gf = 0.0;
    for (int f = f0; f < f1; ++f) {
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
      r_out[q] = (float)r;
      gf += r * b;
    }
    if (accumulate) {
      grad_flat[p] += gf;
    } else {
      const double dfl = (double)flat[p] - mu;
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

// Adjoint seed from stored focal fields (fused evaluation): in place
// Y = w phi G E with G[k][l] = K[k%Q][l%Q] flat[p] r_f[p], p = (k/Q, l/Q);
// per (PSF, row block) FP64 partial of w sum G |E|^2 (the flux gradient).
// With a split output (BF16X3) the seed is written as bf16 hi/lo planes to Ys
// and E is left in place.
template <int SPLIT>
__global__ void seed_kernel(float* Y, long long plane, long long by_psf, int ld, int psf0, int No, int Q, int Nd,
                            int S, int L, const float* sources, const WlInfo* wl, const float* flat, const float* resid,
                            const float* intrapixel, int rows_per_blk, int nblk, double* flux, unsigned short* Ys) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  __shared__ double sh[4];
  const int lb = blockIdx.x / nblk;
  const int blk = blockIdx.x - lb * nblk;
  const int gb = psf0 + lb;
  const int l_idx = gb % L;
  const int fs = gb / L;
  const int f = fs / S;
  const WlInfo wi = wl[l_idx];
  const float wphi = wi.w * sources[fs * 3 + 2];
  const float* rf = resid + (long long)f * Nd * Nd;
  float* yb = Y + (long long)lb * by_psf;
  const int k0 = blk * rows_per_blk;
  const int k1 = min(No, k0 + rows_per_blk);
  const int nq = (No + 3) / 4;                       // groups of 4 columns per row (ld is a multiple of 16)
  const long long n = (long long)(k1 > k0 ? k1 - k0 : 0) * nq;
  double part = 0.0;
  for (long long t = threadIdx.x; t < n; t += blockDim.x) {
    const int k = k0 + (int)(t / nq);
    const int l0 = 4 * (int)(t - (long long)(k - k0) * nq);
    const long long off = (long long)k * ld + l0;
    f4 er = *reinterpret_cast<const f4*>(yb + off);
    f4 ei = *reinterpret_cast<const f4*>(yb + plane + off);
    f4 yr, yi;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int l = l0 + e;
      float g = 0.f;
      if (l < No) {
        const int p = (k / Q) * Nd + (l / Q);
        g = flat[p] * rf[p];
        if (intrapixel) g *= intrapixel[(k % Q) * Q + (l % Q)];
      } else {
        er[e] = 0.f;
        ei[e] = 0.f;
      }
      yr[e] = wphi * g * er[e];
      yi[e] = wphi * g * ei[e];
      part += (double)g * (double)(er[e] * er[e] + ei[e] * ei[e]);
    }
    if constexpr (SPLIT == 0) {
      *reinterpret_cast<f4*>(yb + off) = yr;
      *reinterpret_cast<f4*>(yb + plane + off) = yi;
    } else {
      typedef unsigned short us4 __attribute__((ext_vector_type(4)));
      us4 hr, lr, hi, li;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const __bf16 a = (__bf16)yr[e], b = (__bf16)yi[e];
        hr[e] = __builtin_bit_cast(unsigned short, a);
        lr[e] = __builtin_bit_cast(unsigned short, (__bf16)(yr[e] - (float)a));
        hi[e] = __builtin_bit_cast(unsigned short, b);
        li[e] = __builtin_bit_cast(unsigned short, (__bf16)(yi[e] - (float)b));
      }
      unsigned short* o = Ys + (long long)lb * by_psf + off;
      *reinterpret_cast<us4*>(o) = hr;
      *reinterpret_cast<us4*>(o + plane) = lr;
      *reinterpret_cast<us4*>(o + 2 * plane) = hi;
      *reinterpret_cast<us4*>(o + 3 * plane) = li;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) flux[(long long)gb * nblk + blk] = (double)wi.w * (sh[0] + sh[1] + sh[2] + sh[3]);
}

// gopd[p] = sum_g gpart[g][p]
__global__ void gopd_reduce_kernel(const float* gpart, int G, long long npix, double* gopd) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  double acc = 0.0;
#pragma unroll 8
  for (int g = 0; g < G; ++g) acc += (double)gpart[(long long)g * npix + p];
  gopd[p] = acc;
}

// Zernike projection dL/dc_j = sum_p Z_j[p] gopd[p], in two deterministic passes:
// block (term group of 8, pixel chunk) writes part[chunk][j]; zproj_final sums chunks.
constexpr int kZGroup = 8;

__global__ void zproj_partial_kernel(const float* Z, const double* gopd, int Nz, long long npix, long long chunk,
                                     double* part) {
  __shared__ double sh[4][kZGroup];
  const int j0 = blockIdx.x * kZGroup;
  const long long p_begin = (long long)blockIdx.y * chunk;
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
    part[(long long)blockIdx.y * Nz + j0 + q] = sh[0][q] + sh[1][q] + sh[2][q] + sh[3][q];
  }
}

// one 64-thread wave per term: strided partial sums, then a fixed butterfly
__global__ void zproj_final_kernel(const double* part, int Nz, int nchunks, double* grad) {
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int c = threadIdx.x; c < nchunks; c += 64) acc += part[(long long)c * Nz + j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (threadIdx.x == 0) grad[j] = acc;
}

// tmp2[m][k] = sum_n gopd[m][n] B[n][k]
__global__ void map_grad1_kernel(const double* gopd, const float* Bm, int Ni, int Nmap, double* tmp2) {
  const int m = blockIdx.x;
  const int k = threadIdx.x;
  if (k >= Nmap) return;
  double acc = 0.0;
  for (int n = 0; n < Ni; ++n) acc += gopd[(long long)m * Ni + n] * (double)Bm[(long long)n * Nmap + k];
  tmp2[(long long)m * Nmap + k] = acc;
}

// grad_C[j][k] = sum_m B[m][j] tmp2[m][k]
__global__ void map_grad2_kernel(const double* tmp2, const float* Bm, int Ni, int Nmap, double* grad) {
  const int j = blockIdx.x;
  const int k = threadIdx.x;
  if (k >= Nmap) return;
  double acc = 0.0;
  for (int m = 0; m < Ni; ++m) acc += (double)Bm[(long long)m * Nmap + j] * tmp2[(long long)m * Nmap + k];
  grad[(long long)j * Nmap + k] = acc;
}

// grad_sources[f][s] = (sum over wavelengths and tiles of the position and flux
// partials), one 64-thread block per (frame, star), fixed reduction order.
__global__ void src_reduce_kernel(const double* flux, int tiles_b2, const double* pos, int tiles_b4, int L,
                                  double* grad) {
  __shared__ double sh[3][4];
  const int fs = blockIdx.x;
  const long long b0 = (long long)fs * L;
  double ga = 0.0, gbt = 0.0, gp = 0.0;
  for (int i = threadIdx.x; i < L * tiles_b4; i += 256) {
    const long long q = (b0 * tiles_b4 + i) * 2;
    ga += pos[q];
    gbt += pos[q + 1];
  }
  for (int i = threadIdx.x; i < L * tiles_b2; i += 256) gp += flux[b0 * tiles_b2 + i];
  for (int o = 32; o > 0; o >>= 1) {
    ga += __shfl_xor(ga, o, 64);
    gbt += __shfl_xor(gbt, o, 64);
    gp += __shfl_xor(gp, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = ga;
    sh[1][w] = gbt;
    sh[2][w] = gp;
  }
  __syncthreads();
  if (threadIdx.x < 3) grad[fs * 3 + threadIdx.x] = sh[threadIdx.x][0] + sh[threadIdx.x][1] + sh[threadIdx.x][2] + sh[threadIdx.x][3];
}

}  // namespace

hipError_t launch_intensity(dlx_plan* p, int f0, int nf, const float* sources, const float* intrapixel,
                            const float* flat, float* binned, float* model, hipStream_t st) {
  const long long npix = (long long)p->Nd * p->Nd;
  const dim3 grid((unsigned)((npix + 63) / 64), nf), blk(64, 4);
  const long long plane = (long long)p->chunk_psf * p->No * p->ldNo, by = (long long)p->No * p->ldNo;
#define DLX_INTENSITY(QT)                                                                                         \
  hipLaunchKernelGGL(intensity_kernel<QT>, grid, blk, 0, st, p->d_Y, plane, by, p->ldNo, f0, p->F, p->S, p->L, \
                     p->Q, p->Nd, sources, p->d_wl, intrapixel, flat, binned, model)
  switch (p->Q) {
    case 2: DLX_INTENSITY(2); break;
    case 4: DLX_INTENSITY(4); break;
    default: DLX_INTENSITY(0); break;
  }
#undef DLX_INTENSITY
  return hipGetLastError();
}

hipError_t launch_seed(dlx_plan* p, int f0, int nf, const float* sources, const float* flat, const float* resid,
                       const float* intrapixel, hipStream_t st) {
  const int nc = nf * p->S * p->L;
  const int nblk = p->tiles_b2;
  const int rows = (p->No + nblk - 1) / nblk;
  const long long plane = (long long)p->chunk_psf * p->No * p->ldNo, by = (long long)p->No * p->ldNo;
  if (p->bf16())
    hipLaunchKernelGGL(seed_kernel<1>, dim3(nc * nblk), dim3(256), 0, st, p->d_Y, plane, by, p->ldNo,
                       f0 * p->S * p->L, p->No, p->Q, p->Nd, p->S, p->L, sources, p->d_wl, flat, resid, intrapixel,
                       rows, nblk, p->d_flux, static_cast<unsigned short*>(p->d_Ys));
  else
    hipLaunchKernelGGL(seed_kernel<0>, dim3(nc * nblk), dim3(256), 0, st, p->d_Y, plane, by, p->ldNo,
                       f0 * p->S * p->L, p->No, p->Q, p->Nd, p->S, p->L, sources, p->d_wl, flat, resid, intrapixel,
                       rows, nblk, p->d_flux, nullptr);
  return hipGetLastError();
}

int loss_block_count(long long npix) { return (int)((npix + kLossThreads - 1) / kLossThreads); }

// Loss terms of frames [f0, f0 + nf); block partials at slot `chunk`. The
// loss itself is summed by launch_loss_final over `n_chunks` slots.
hipError_t launch_loss(dlx_plan* p, int f0, int nf, int chunk, const float* model, const float* binned,
                       const float* data, const float* flat, int kind, double mu, double sigma, float* r, double* gflat,
                       hipStream_t st) {
  const long long npix = (long long)p->Nd * p->Nd;
  const int nb = loss_block_count(npix);
  hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(kLossThreads), 0, st, model, binned, data, flat, f0, f0 + nf, npix,
                     kind, mu, 1.0 / (sigma * sigma), r, gflat, chunk > 0 ? 1 : 0, p->d_lossblk + (long long)chunk * nb,
                     p->d_status);
  return hipGetLastError();
}

hipError_t launch_loss_final(dlx_plan* p, int n_chunks, double* loss, hipStream_t st) {
  const int nb = loss_block_count((long long)p->Nd * p->Nd);
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(1024), 0, st, p->d_lossblk, nb * n_chunks, loss);
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

hipError_t launch_grad_reduce(dlx_plan* p, const float* Z, const float* Bm, double* gz, double* gmap, double* gsrc,
                              hipStream_t st) {
  const long long npix = (long long)p->Ni * p->Ni;
  const int G = p->b4_groups_max * p->b4_ksplit;
  hipLaunchKernelGGL(gopd_reduce_kernel, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, p->d_gpart, G, npix,
                     p->d_gopd);
  if (p->Nz > 0) {
    const int nch = zproj_chunks(npix, p->Nz);
    const long long chunk = ((npix + nch - 1) / nch + 1023) / 1024 * 1024;
    hipLaunchKernelGGL(zproj_partial_kernel, dim3((p->Nz + kZGroup - 1) / kZGroup, nch), dim3(256), 0, st, Z,
                       p->d_gopd, p->Nz, npix, chunk, p->d_zpart);
    hipLaunchKernelGGL(zproj_final_kernel, dim3(p->Nz), dim3(64), 0, st, p->d_zpart, p->Nz, nch, gz);
  }
  if (p->Nmap > 0) {
    hipLaunchKernelGGL(map_grad1_kernel, dim3(p->Ni), dim3((p->Nmap + 63) / 64 * 64), 0, st, p->d_gopd, Bm, p->Ni,
                       p->Nmap, p->d_tmp2);
    hipLaunchKernelGGL(map_grad2_kernel, dim3(p->Nmap), dim3((p->Nmap + 63) / 64 * 64), 0, st, p->d_tmp2, Bm, p->Ni,
                       p->Nmap, gmap);
  }
  hipLaunchKernelGGL(src_reduce_kernel, dim3(p->F * p->S), dim3(256), 0, st, p->d_flux, p->tiles_b2, p->d_pos,
                     p->tiles_b4 * p->b4_ksplit, p->L, gsrc);
  return hipGetLastError();
}

}  // namespace dlx
