// Operand preparation for the two-sided MFT (Section 3).
//
//   DFT matrices   M_l[k][n] = exp(-2 pi i x_n u_k / lambda_l), stored once per plan as
//                  M (rows = focal index) and M^T (rows = pupil index), planar FP32, or
//                  split into bf16 hi/lo planes from the FP64 value (BF16X3 plans).
//                  x_n u_k / lambda = (2n - Ni + 1)(2k - No + 1) * dx du / (4 lambda):
//                  the integer product is exact, the scale is FP64 and the result is
//                  reduced modulo one cycle before sincospi, so the phase error does
//                  not grow with the grid size.
//   OPD            sum_j c_j Z_j (+ B C B^T), FP64 accumulation split over term groups (basis optic, Section 3).
//   Pupil field    P0_l = A / sqrt(sum A^2) * exp(i 2 pi OPD / lambda_l), stored transposed.
//   Tilts          tx[n] = exp(+2 pi i x_n alpha / lambda), ty[m] likewise with beta,
//                  one pair of vectors per PSF, phases in FP64 reduced modulo one cycle.
// All of these are HBM- or launch-bound; none is on the MFMA path.
#include "dlx_internal.h"

namespace dlx {
namespace {

// Split of an FP64 value into bf16 hi (RNE of the FP32 rounding) and lo (RNE of the rest).
__device__ __forceinline__ void split64(double x, unsigned short& hi, unsigned short& lo) {
  const __bf16 h = (__bf16)(float)x;
  const __bf16 l = (__bf16)(float)(x - (double)(float)h);
  hi = __builtin_bit_cast(unsigned short, h);
  lo = __builtin_bit_cast(unsigned short, l);
}

template <int SPLIT>
__device__ __forceinline__ void put_m(void* base, long long plane, long long idx, double re, double im) {
  if constexpr (SPLIT == 0) {
    float* o = static_cast<float*>(base);
    o[idx] = (float)re;
    o[plane + idx] = (float)im;
  } else {
    unsigned short* o = static_cast<unsigned short*>(base);
    unsigned short h, l;
    split64(re, h, l);
    o[idx] = h;
    o[plane + idx] = l;
    split64(im, h, l);
    o[2 * plane + idx] = h;
    o[3 * plane + idx] = l;
  }
}

template <int SPLIT>
__global__ void dft_matrix_kernel(void* MN, void* MT, int Ni, int No, int ldNi, int ldNo, double s4,
                                  const WlInfo* wl, long long mn_plane, long long mn_wl, long long mt_plane,
                                  long long mt_wl) {
  const int l = blockIdx.z;
  const double s = s4 / wl[l].lam;  // dx du / (4 lambda)
  const int n = blockIdx.x * blockDim.x + threadIdx.x;  // pupil index (padded)
  const int k = blockIdx.y * blockDim.y + threadIdx.y;  // focal index (padded)
  if (n >= ldNi && n >= Ni) return;
  double re = 0.0, im = 0.0;
  if (n < Ni && k < No) {
    const long long p = (long long)(2 * n - Ni + 1) * (long long)(2 * k - No + 1);
    const double t = (double)p * s;           // cycles
    const double fr = t - rint(t);
    double sn, cs;
    sincospi(2.0 * fr, &sn, &cs);
    re = cs;
    im = -sn;
  }
  if (k < No && n < ldNi) put_m<SPLIT>(MN, mn_plane, l * mn_wl + (long long)k * ldNi + n, re, im);
  if (n < Ni && k < ldNo) put_m<SPLIT>(MT, mt_plane, l * mt_wl + (long long)n * ldNo + k, re, im);
}

// Coordinates of the pupil samples (x and y grids are identical).
__global__ void coords_kernel(double* x, int Ni, double dx) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < Ni) x[n] = ((double)n - 0.5 * (double)(Ni - 1)) * dx;
}

// tmp[j][n] = sum_k C[j][k] B[n][k]   (first half of B C B^T)
__global__ void map_tmp_kernel(const float* C, const float* Bm, float* tmp, int Nmap, int Ni) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (n >= Ni) return;
  double acc = 0.0;
  for (int k = 0; k < Nmap; ++k) acc += (double)C[j * Nmap + k] * (double)Bm[(long long)n * Nmap + k];
  tmp[(long long)j * Ni + n] = (float)acc;
}

// P0T_l[n][m] = A[m][n] / sqrt(sum A^2) * exp(i 2 pi OPD[m][n] / lambda_l), one block per
// (32 x 32 tile, nl consecutive wavelengths from l0), transposed through LDS; the tile's OPD,
// screen and transmission are read once for all of its wavelengths. Row n stores column m at m for
// m < h and at m + ldp - Ni for h <= m < Ni (the folded layout; h = Ni: natural), zeros elsewhere.
template <int NLMAX>   // nl <= NLMAX (1: the single-wavelength body, with no loop state)
__device__ __forceinline__ void pupil_body(int bx, int by, int l0, int nl, int L, const float* A, const double* opd,
                                           const float* screen, const double* norm_part, int n_norm,
                                           const WlInfo* wl, int Ni, int ldp, int h, float* P0T, long long plane,
                                           long long by_wl) {
  __shared__ float tr[32][33], ti[32][33];
  __shared__ double sparts[256];   // n_norm <= 256
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  const int m0 = by * 32, n0 = bx * 32;
  // the partial sums of A^2 are read in parallel, next to the pixels' loads
  for (int i = ty * 32 + tx; i < n_norm; i += 256) sparts[i] = norm_part[i];
  double od[4], sc[4], av[4];
  bool in[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = m0 + ty + 8 * q, n = n0 + tx;
    in[q] = m < Ni && n < Ni;
    od[q] = sc[q] = av[q] = 0.0;
    if (in[q]) {
      const long long p = (long long)m * Ni + n;
      od[q] = opd[p];
      sc[q] = (double)screen[p] * 0.15915494309189533577;   // the static screen in cycles (achromatic)
      av[q] = (double)A[p];
    }
  }
  __syncthreads();
  double s2 = 0.0;   // every thread adds the partials in the same order
  for (int i = 0; i < n_norm; ++i) s2 += sparts[i];
  const double nrm = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
  const int l_end = l0 + nl < L ? l0 + nl : L;
#pragma unroll
  for (int i = 0; i < NLMAX; ++i) {
    const int l = l0 + i;
    if (l >= l_end) break;
    const double inv = 1.0 / wl[l].lam;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double sn = 0.0, cs = 0.0;
      if (in[q]) {
        const double t0 = od[q] * inv + sc[q];   // phase in cycles
        const double fr = t0 - rint(t0);
        sincospi(2.0 * fr, &sn, &cs);
      }
      const double amp = av[q] * nrm;
      tr[ty + 8 * q][tx] = (float)(amp * cs);
      ti[ty + 8 * q][tx] = (float)(amp * sn);
    }
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int n = n0 + ty + 8 * q, m = m0 + tx;  // output row n, column m
      if (n < Ni && m < ldp) {
        const bool inside = m < Ni;
        // the ldp - Ni padding columns m >= Ni fill the gap [h, h + ldp - Ni)
        const int c = m < h ? m : (inside ? m + (ldp - Ni) : h + (m - Ni));
        P0T[l * by_wl + (long long)n * ldp + c] = inside ? tr[tx][ty + 8 * q] : 0.f;
        P0T[l * by_wl + plane + (long long)n * ldp + c] = inside ? ti[tx][ty + 8 * q] : 0.f;
      }
    }
    if (i + 1 < NLMAX && l + 1 < l_end) __syncthreads();   // the next wavelength rewrites the tile
  }
}

template <int NLMAX>
__global__ __launch_bounds__(256) void pupil_kernel(const float* A, const double* opd, const float* screen,
                                                    const double* norm_part, int n_norm, const WlInfo* wl, int Ni,
                                                    int ldp, int h, float* P0T, long long plane, long long by_wl,
                                                    int nl, int L) {
  pupil_body<NLMAX>(blockIdx.x, blockIdx.y, blockIdx.z * nl, nl, L, A, opd, screen, norm_part, n_norm, wl, Ni, ldp, h,
                    P0T, plane, by_wl);
}

// The pupil fields of every problem of a multi-problem plan in one launch (block table entries:
// problem, tile column, tile row, first wavelength; kPupilGroupWl wavelengths per block).
__global__ __launch_bounds__(256) void pupil_group_kernel(const PupilArgs* __restrict__ args,
                                                          const GroupBlock* __restrict__ tab, const float* A) {
  const GroupBlock e = tab[blockIdx.x];
  const PupilArgs& a = args[e.k];
  pupil_body<kPupilGroupWl>(e.x, e.y, e.z, kPupilGroupWl, a.L, A + a.o_trans, a.opd, a.screen, a.norm_part, a.n_norm, a.wl, a.Ni,
             a.ldp, a.h, a.P0T, a.plane, a.by_wl);
}

// Tilt vectors of all PSFs, psf = (f S + s) L + l: element t = psf * ldt + n.
__device__ void tilt_at(long long t, const float* sources, const WlInfo* wl, const double* x, int L, int Ni, int ldt,
                        float* tx, float* ty, long long plane) {
  const int gb = (int)(t / ldt);
  const int n = (int)(t - (long long)gb * ldt);
  const int l = gb % L;
  const int fs = gb / L;  // f * S + s
  const double alpha = sources[fs * 3 + 0], beta = sources[fs * 3 + 1];
  float xr = 0.f, xi = 0.f, yr = 0.f, yi = 0.f;
  if (n < Ni) {
    const double inv = 1.0 / wl[l].lam;
    double sn, cs;
    double u = x[n] * alpha * inv;
    u -= rint(u);
    sincospi(2.0 * u, &sn, &cs);
    xr = (float)cs;
    xi = (float)sn;
    u = x[n] * beta * inv;
    u -= rint(u);
    sincospi(2.0 * u, &sn, &cs);
    yr = (float)cs;
    yi = (float)sn;
  }
  tx[t] = xr;
  tx[plane + t] = xi;
  ty[t] = yr;
  ty[plane + t] = yi;
}

// The parameter-dependent inputs of the MFT in one launch (256 threads),
// three independent jobs by block range:
//   [0, nb_opd):              OPD[p] = sum_j c_j Z_j[p] (+ sum_j B[m][j] tmp[j][n]),
//                             one pixel per thread, FP64 accumulation in term order;
//   [nb_opd, nb_opd + n_norm): partial sums of A^2 (grid-stride over the pixels),
//                             one per block, added by the pupil kernel in order;
//   the rest:                 the tilt vectors tx, ty of every PSF.
__device__ __forceinline__ void prep_body(int b, const float* Z, const float* c, int Nz, long long npix, int Ni,
                                          const float* Bm, const float* tmp, int Nmap, double* opd, int nb_opd,
                                          const float* A, double* norm_part, int n_norm, const float* sources,
                                          const WlInfo* wl, const double* x, int L, int ldt, long long n_tilt,
                                          float* tx, float* ty, long long tplane) {
  if (b < nb_opd) {
    const long long p = (long long)b * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    double acc = 0.0;
    const float* z = Z + p;
    int j = 0;
    for (; j + 8 <= Nz; j += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = z[(long long)(j + u) * npix];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += (double)c[j + u] * (double)v[u];
    }
    for (; j < Nz; ++j) acc += (double)c[j] * (double)z[(long long)j * npix];
    if (Nmap > 0) {
      const int m = (int)(p / Ni), n = (int)(p - (long long)m * Ni);
      double a = 0.0;
      for (int k = 0; k < Nmap; ++k) a += (double)Bm[(long long)m * Nmap + k] * (double)tmp[(long long)k * Ni + n];
      acc += a;
    }
    opd[p] = acc;
  } else if (b < nb_opd + n_norm) {
    __shared__ double sh[4];
    const int nb = b - nb_opd;
    double acc = 0.0;
    for (long long i = (long long)nb * blockDim.x + threadIdx.x; i < npix; i += (long long)n_norm * blockDim.x) {
      const double v = A[i];
      acc += v * v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) norm_part[nb] = sh[0] + sh[1] + sh[2] + sh[3];
  } else {
    const long long t = (long long)(b - nb_opd - n_norm) * blockDim.x + threadIdx.x;
    if (t < n_tilt) tilt_at(t, sources, wl, x, L, Ni, ldt, tx, ty, tplane);
  }
}

__global__ __launch_bounds__(256) void prep_kernel(const float* Z, const float* c, int Nz, long long npix, int Ni,
                                                   const float* Bm, const float* tmp, int Nmap, double* opd,
                                                   int nb_opd, const float* A, double* norm_part, int n_norm,
                                                   const float* sources, const WlInfo* wl, const double* x, int L,
                                                   int ldt, long long n_tilt, float* tx, float* ty, long long tplane) {
  prep_body(blockIdx.x, Z, c, Nz, npix, Ni, Bm, tmp, Nmap, opd, nb_opd, A, norm_part, n_norm, sources, wl, x, L, ldt,
            n_tilt, tx, ty, tplane);
}

// prep_kernel's three jobs for every problem of a multi-problem plan in one launch (block table
// entries: problem, block of that problem's prep grid); no bicubic map.
__global__ __launch_bounds__(256) void prep_group_kernel(const PrepArgs* __restrict__ args,
                                                         const GroupBlock* __restrict__ tab, GroupCall call) {
  const GroupBlock e = tab[blockIdx.x];
  const PrepArgs& a = args[e.k];
  prep_body(e.x, a.Nz ? call.zbasis + a.o_z : nullptr, a.Nz ? call.coeffs + a.o_c : nullptr, a.Nz, a.npix, a.Ni,
            nullptr, nullptr, 0, a.opd, a.nb_opd, call.transmission + a.o_trans, a.norm_part, a.n_norm,
            call.sources + a.o_src, a.wl, a.x, a.L, a.ldt, a.n_tilt, a.tx, a.ty, a.tplane);
}

}  // namespace

hipError_t launch_dft(dlx_plan* p, hipStream_t st) {
  const dim3 blk(64, 4);
  const int nmax = p->ldNi > p->Ni ? p->ldNi : p->Ni;
  const int kmax = p->ldNo > p->No ? p->ldNo : p->No;
  const dim3 grid((nmax + 63) / 64, (kmax + 3) / 4, p->L);
  const long long mn_plane = (long long)p->L * p->No * p->ldNi;
  const long long mt_plane = (long long)p->L * p->Ni * p->ldNo;
  const double s4 = p->dx * p->du / 4.0;
  if (p->bf16())
    hipLaunchKernelGGL(dft_matrix_kernel<1>, grid, blk, 0, st, p->d_MN, p->d_MT, p->Ni, p->No, p->ldNi, p->ldNo, s4,
                       p->d_wl, mn_plane, (long long)p->No * p->ldNi, mt_plane, (long long)p->Ni * p->ldNo);
  else
    hipLaunchKernelGGL(dft_matrix_kernel<0>, grid, blk, 0, st, p->d_MN, p->d_MT, p->Ni, p->No, p->ldNi, p->ldNo, s4,
                       p->d_wl, mn_plane, (long long)p->No * p->ldNi, mt_plane, (long long)p->Ni * p->ldNo);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(coords_kernel, dim3((p->Ni + 255) / 256), dim3(256), 0, st, p->d_x, p->Ni, p->dx);
  return hipGetLastError();
}

__global__ void zero_kernel(float* x, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.f;
}

hipError_t launch_zero(float* x, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n);
  return hipGetLastError();
}

hipError_t launch_prep(dlx_plan* p, const float* A, const float* Z, const float* Bm, const float* c, const float* C,
                       const float* sources, hipStream_t st) {
  const long long npix = (long long)p->Ni * p->Ni;
  if (p->Nmap > 0) {
    hipLaunchKernelGGL(map_tmp_kernel, dim3((p->Ni + 255) / 256, p->Nmap), dim3(256), 0, st, C, Bm, p->d_maptmp,
                       p->Nmap, p->Ni);
  }
  const int nb_opd = (int)((npix + 255) / 256);
  const long long nt = (long long)p->n_psf * p->ldNi;
  const int nb_tilt = (int)((nt + 255) / 256);
  hipLaunchKernelGGL(prep_kernel, dim3(nb_opd + p->n_norm_part + nb_tilt), dim3(256), 0, st, Z, c, p->Nz, npix, p->Ni,
                     Bm, p->d_maptmp, p->Nmap, p->d_opd, nb_opd, A, p->d_norm, p->n_norm_part, sources, p->d_wl,
                     p->d_x, p->L, p->ldNi, nt, p->d_tx, p->d_ty, nt);
  const long long p0_by_wl = 2LL * p->Ni * p->ldNi;
  // wavelengths per block: up to 8 (each tile's loads and norm serve them all) while the launch
  // keeps at least 2048 blocks
  const long long tiles = (long long)((p->Ni + 31) / 32) * ((p->ldNi + 31) / 32);
  int nl = 8;
  while (nl > 1 && tiles * ((p->L + nl - 1) / nl) < 2048) nl /= 2;
  const dim3 pgrid((p->Ni + 31) / 32, (p->ldNi + 31) / 32, (p->L + nl - 1) / nl);
  if (nl == 1)
    hipLaunchKernelGGL(pupil_kernel<1>, pgrid, dim3(32, 8), 0, st, A, p->d_opd, p->d_screen, p->d_norm,
                       p->n_norm_part, p->d_wl, p->Ni, p->ldNi, p->fold ? p->hNi() : p->Ni, p->d_P0T,
                       (long long)p->Ni * p->ldNi, p0_by_wl, nl, p->L);
  else
    hipLaunchKernelGGL(pupil_kernel<8>, pgrid, dim3(32, 8), 0, st, A, p->d_opd, p->d_screen, p->d_norm,
                       p->n_norm_part, p->d_wl, p->Ni, p->ldNi, p->fold ? p->hNi() : p->Ni, p->d_P0T,
                       (long long)p->Ni * p->ldNi, p0_by_wl, nl, p->L);
  return hipGetLastError();
}

hipError_t launch_prep_group(const PrepArgs* args, const GroupBlock* tab, int n_blocks, const GroupCall& call,
                             hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(prep_group_kernel, dim3(n_blocks), dim3(256), 0, st, args, tab, call);
  return hipGetLastError();
}

hipError_t launch_pupil_group(const PupilArgs* args, const GroupBlock* tab, int n_blocks, const GroupCall& call,
                              hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(pupil_group_kernel, dim3(n_blocks), dim3(32, 8), 0, st, args, tab, call.transmission);
  return hipGetLastError();
}

}  // namespace dlx
