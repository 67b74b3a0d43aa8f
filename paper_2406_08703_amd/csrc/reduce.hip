// HBM-bound stages around the MFT: group reduction of binned partials and
// the pixel response (Section 3), the Poisson / chi-squared loss with the
// pixel-response prior and its gradients (Section 4), and the projections of
// dL/dOPD onto the Zernike basis and the bicubic map. Every reduction runs in
// FP64 in a fixed order, so results are bitwise reproducible.
#include "dlx_internal.h"

namespace dlx {
namespace {

// binned[f][p] = sum_g part[f][g][p];  model[f][p] = flat[p] * binned[f][p]
__global__ void bin_reduce_kernel(const float* part, int G, int F, long long npix, const float* flat, float* binned,
                                  float* model) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (p >= npix || f >= F) return;
  const float* src = part + (long long)f * G * npix + p;
  double acc = 0.0;
  for (int g = 0; g < G; ++g) acc += (double)src[(long long)g * npix];
  const float b = (float)acc;
  binned[(long long)f * npix + p] = b;
  model[(long long)f * npix + p] = flat[p] * b;
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

// Per pixel p: loop over frames, l = m - d ln m (or (m-d)^2/(2 max(d,1))),
// r = dl/dm, grad_flat[p] = sum_f r B + (F - mu)/sigma^2; block partial of L.
__global__ void loss_kernel(const float* model, const float* binned, const float* data, const float* flat, int F,
                            long long npix, int kind, double mu, double inv_s2, float* r_out, double* grad_flat,
                            double* blk, int* status) {
  __shared__ double sh[kLossThreads / 64];
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double lsum = 0.0;
  int flags = 0;
  if (p < npix) {
    double gf = 0.0;
    for (int f = 0; f < F; ++f) {
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
    const double fl = flat[p];
    const double dfl = fl - mu;
    lsum += 0.5 * dfl * dfl * inv_s2;
    grad_flat[p] = gf + dfl * inv_s2;
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

// gopd[p] = sum_g gpart[g][p]
__global__ void gopd_reduce_kernel(const float* gpart, int G, long long npix, double* gopd) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  double acc = 0.0;
  for (int g = 0; g < G; ++g) acc += (double)gpart[(long long)g * npix + p];
  gopd[p] = acc;
}

// grad_c[j] = sum_p Z_j[p] gopd[p]: one block per term.
__global__ void zproj_kernel(const float* Z, const double* gopd, long long npix, double* grad) {
  __shared__ double sh[512 / 64];
  const int j = blockIdx.x;
  const float* z = Z + (long long)j * npix;
  double acc = 0.0;
  for (long long p = threadIdx.x; p < npix; p += blockDim.x) acc += (double)z[p] * gopd[p];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) grad[j] = t;
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

// grad_sources[f][s] = (sum_l sum_tiles pos, sum_l sum_tiles flux)
__global__ void src_reduce_kernel(const double* flux, int tiles_b2, const double* pos, int tiles_b4, int FS, int L,
                                  double* grad) {
  const int fs = blockIdx.x * blockDim.x + threadIdx.x;
  if (fs >= FS) return;
  double ga = 0.0, gbt = 0.0, gp = 0.0;
  for (int l = 0; l < L; ++l) {
    const long long b = (long long)fs * L + l;
    for (int t = 0; t < tiles_b4; ++t) {
      ga += pos[(b * tiles_b4 + t) * 2 + 0];
      gbt += pos[(b * tiles_b4 + t) * 2 + 1];
    }
    for (int t = 0; t < tiles_b2; ++t) gp += flux[b * tiles_b2 + t];
  }
  grad[fs * 3 + 0] = ga;
  grad[fs * 3 + 1] = gbt;
  grad[fs * 3 + 2] = gp;
}

}  // namespace

hipError_t launch_bin_reduce(dlx_plan* p, const float* flat, float* binned, float* model, hipStream_t st) {
  const long long npix = (long long)p->Nd * p->Nd;
  hipLaunchKernelGGL(bin_reduce_kernel, dim3((unsigned)((npix + 255) / 256), p->F), dim3(256), 0, st, p->d_binpart,
                     p->f2_groups, p->F, npix, flat, binned, model);
  return hipGetLastError();
}

int loss_block_count(long long npix) { return (int)((npix + kLossThreads - 1) / kLossThreads); }

hipError_t launch_loss(dlx_plan* p, const float* model, const float* binned, const float* data, const float* flat,
                       int kind, double mu, double sigma, double* loss, float* r, double* gflat, hipStream_t st) {
  const long long npix = (long long)p->Nd * p->Nd;
  const int nb = loss_block_count(npix);
  hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(kLossThreads), 0, st, model, binned, data, flat, p->F, npix, kind,
                     mu, 1.0 / (sigma * sigma), r, gflat, p->d_lossblk, p->d_status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(1024), 0, st, p->d_lossblk, nb, loss);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(dlx_plan* p, const float* Z, const float* Bm, double* gz, double* gmap, double* gsrc,
                              hipStream_t st) {
  const long long npix = (long long)p->Ni * p->Ni;
  const int G = p->b4_groups_max;
  hipLaunchKernelGGL(gopd_reduce_kernel, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, p->d_gpart, G, npix,
                     p->d_gopd);
  if (p->Nz > 0)
    hipLaunchKernelGGL(zproj_kernel, dim3(p->Nz), dim3(512), 0, st, Z, p->d_gopd, npix, gz);
  if (p->Nmap > 0) {
    hipLaunchKernelGGL(map_grad1_kernel, dim3(p->Ni), dim3((p->Nmap + 63) / 64 * 64), 0, st, p->d_gopd, Bm, p->Ni,
                       p->Nmap, p->d_tmp2);
    hipLaunchKernelGGL(map_grad2_kernel, dim3(p->Nmap), dim3((p->Nmap + 63) / 64 * 64), 0, st, p->d_tmp2, Bm, p->Ni,
                       p->Nmap, gmap);
  }
  const int FS = p->F * p->S;
  hipLaunchKernelGGL(src_reduce_kernel, dim3((FS + 127) / 128), dim3(128), 0, st, p->d_flux, p->tiles_b2, p->d_pos,
                     p->tiles_b4, FS, p->L, gsrc);
  return hipGetLastError();
}

}  // namespace dlx
