// Batched planar-complex GEMMs of the two-sided matrix Fourier transform
// (Section 3: one product per side of the MFT) and of its adjoint, on FP32
// MFMA (v_mfma_f32_16x16x4_f32) for gfx950.
//
// Every stage is a "TN" product C[i][j] = sum_k A[i][k] B[j][k] with both
// operands K-contiguous, so one 128-bit LDS read feeds four MFMA k-steps.
// A workgroup of 4 waves (2 x 2) owns a (32 WM) x (32 WN) complex output
// tile; each wave holds WM x WN 16 x 16 blocks of real and imaginary
// accumulators. K advances 16 at a time through one LDS stage, with the next
// stage's global loads in flight during the MFMAs.
//
// The complex product uses the four real products Re = ArBr - AiBi,
// Im = ArBi + AiBr (no 3-multiply trick: it loses accuracy on operands of
// very different size). Operand conjugation negates the imaginary part on
// load. Stage-specific work is fused into the operand loader (the pupil
// field of F1 is generated from P0^T, the row tilt and the column tilt) and
// into the epilogues (intensity, intra-pixel weighting and binning for F2;
// the adjoint seed for B2; the phase gradient and position sums for B4).
#include "dlx_internal.h"

namespace dlx {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
// that a contiguous range of logical ids (same PSF / same wavelength, whose
// operands are shared) runs on one XCD and reuses its L2.
__device__ __forceinline__ int xcd_remap(int w, int n) {
  const int q = n >> 3, r = n & 7;
  const int xcd = w & 7, k = w >> 3;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + k;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int KIND, int WM, int WN>
__global__ __launch_bounds__(256) void cgemm_kernel(const GemmArgs a) {
  constexpr int BM = 32 * WM, BN = 32 * WN, BK = 16, LDK = 20;
  constexpr int A_FL = 2 * BM * LDK, B_FL = 2 * BN * LDK;
  constexpr int OPS_FL = A_FL + B_FL;
  constexpr int EPI_FL = (KIND == KIND_F2) ? BM * BN : 0;
  constexpr int SM_FL = OPS_FL > EPI_FL ? OPS_FL : EPI_FL;
  constexpr int A_PAIRS = (BM * 4 + 255) / 256;
  constexpr int B_PAIRS = (BN * 4 + 255) / 256;
  __shared__ __attribute__((aligned(16))) float smem[SM_FL];
  __shared__ double sred[8];
  float* As = smem;
  float* Bs = smem + A_FL;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int tiles = a.tiles_m * a.tiles_n;
  const int item = lin / tiles;
  if (item >= a.n_items) return;
  const int tile = lin - item * tiles;
  const int tm = tile / a.tiles_n, tn = tile - tm * a.tiles_n;
  const int row0 = tm * BM, col0 = tn * BN;
  const int M = a.M, N = a.N, K = a.K;

  int p_begin, p_end, grp = 0, fl = 0;
  if constexpr (KIND == KIND_F2) {
    fl = item / a.groups;
    grp = item - fl * a.groups;
    const int base = fl * a.S * a.L;
    p_begin = base + grp * a.group_size;
    p_end = min(p_begin + a.group_size, base + a.S * a.L);
  } else if constexpr (KIND == KIND_B4) {
    grp = item;
    const int g = item / a.ksplit;
    p_begin = g * a.group_size;
    p_end = min(p_begin + a.group_size, a.n_chunk_psf);
  } else {
    p_begin = item;
    p_end = item + 1;
  }

  f4 sum[WM][WN];
#pragma unroll
  for (int bm = 0; bm < WM; ++bm)
#pragma unroll
    for (int bn = 0; bn < WN; ++bn) sum[bm][bn] = f4{0.f, 0.f, 0.f, 0.f};

  // K range of this item (split only for B4, whose epilogue is linear in the product)
  int k_lo = 0, k_hi = K;
  if constexpr (KIND == KIND_B4) {
    const int ks = item % a.ksplit;
    const int kc = ((K + a.ksplit * BK - 1) / (a.ksplit * BK)) * BK;
    k_lo = ks * kc;
    k_hi = min(K, k_lo + kc);
  }
  const int nk = k_hi > k_lo ? (k_hi - k_lo + BK - 1) / BK : 0;

  for (int lb = p_begin; lb < p_end; ++lb) {
    const int gb = a.psf0 + lb;
    const int wl = gb % a.L;
    const float* Ab = a.A.base + (long long)wl * a.A.by_wl + (long long)lb * a.A.by_psf;
    const float* Bb = a.B.base + (long long)wl * a.B.by_wl + (long long)lb * a.B.by_psf;
    const float* txb = a.tx + (long long)gb * a.ldt;
    const float* tyb = a.ty + (long long)gb * a.ldt;

    f4 accr[WM][WN], acci[WM][WN];
#pragma unroll
    for (int bm = 0; bm < WM; ++bm)
#pragma unroll
      for (int bn = 0; bn < WN; ++bn) {
        accr[bm][bn] = f4{0.f, 0.f, 0.f, 0.f};
        acci[bm][bn] = f4{0.f, 0.f, 0.f, 0.f};
      }

    // Raw global loads of the next K tile. They are consumed only by
    // store_tile (after the MFMAs), so their latency overlaps the MFMAs:
    // conjugation, K-tail masking and the F1 pupil-field product are applied
    // at store time, never right after the load.
    f4 ga_r[A_PAIRS], ga_i[A_PAIRS], gb_r[B_PAIRS], gb_i[B_PAIRS];
    f4 gy_r[B_PAIRS], gy_i[B_PAIRS];
    float gx_r[B_PAIRS], gx_i[B_PAIRS];
    int ga_k[A_PAIRS], gb_k[B_PAIRS];

    auto load_tile = [&](int k0) {
#pragma unroll
      for (int r = 0; r < A_PAIRS; ++r) {
        const int q = tid + 256 * r;
        const int row = q >> 2, kq = q & 3;
        const int gi = row0 + row, gk = k0 + 4 * kq;
        ga_k[r] = gk;
        ga_r[r] = f4{0.f, 0.f, 0.f, 0.f};
        ga_i[r] = ga_r[r];
        if (q < BM * 4 && gi < M && gk < k_hi) {
          const float* p = Ab + (long long)gi * a.A.ld + gk;
          ga_r[r] = *reinterpret_cast<const f4*>(p);
          ga_i[r] = *reinterpret_cast<const f4*>(p + a.A.plane);
        }
      }
#pragma unroll
      for (int r = 0; r < B_PAIRS; ++r) {
        const int q = tid + 256 * r;
        const int row = q >> 2, kq = q & 3;
        const int gj = col0 + row, gk = k0 + 4 * kq;
        gb_k[r] = gk;
        gb_r[r] = f4{0.f, 0.f, 0.f, 0.f};
        gb_i[r] = gb_r[r];
        if constexpr (KIND == KIND_F1) {
          gy_r[r] = gb_r[r];
          gy_i[r] = gb_r[r];
          gx_r[r] = 0.f;
          gx_i[r] = 0.f;
        }
        if (q < BN * 4 && gj < N && gk < k_hi) {
          const float* p = Bb + (long long)gj * a.B.ld + gk;
          gb_r[r] = *reinterpret_cast<const f4*>(p);
          gb_i[r] = *reinterpret_cast<const f4*>(p + a.B.plane);
          if constexpr (KIND == KIND_F1) {
            gy_r[r] = *reinterpret_cast<const f4*>(tyb + gk);
            gy_i[r] = *reinterpret_cast<const f4*>(tyb + a.tilt_plane + gk);
            gx_r[r] = txb[gj];
            gx_i[r] = txb[a.tilt_plane + gj];
          }
        }
      }
    };

    auto fix = [&](f4& vr, f4& vi, int gk, bool conj) {
      if (gk + 4 > k_hi) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (gk + e >= k_hi) {
            vr[e] = 0.f;
            vi[e] = 0.f;
          }
      }
      if (conj) vi = -vi;
    };

    auto store_tile = [&]() {
#pragma unroll
      for (int r = 0; r < A_PAIRS; ++r) {
        const int q = tid + 256 * r;
        if (q < BM * 4) {
          const int row = q >> 2, kq = q & 3;
          f4 vr = ga_r[r], vi = ga_i[r];
          fix(vr, vi, ga_k[r], a.conj_a);
          *reinterpret_cast<f4*>(&As[row * LDK + 4 * kq]) = vr;
          *reinterpret_cast<f4*>(&As[(BM + row) * LDK + 4 * kq]) = vi;
        }
      }
#pragma unroll
      for (int r = 0; r < B_PAIRS; ++r) {
        const int q = tid + 256 * r;
        if (q < BN * 4) {
          const int row = q >> 2, kq = q & 3;
          f4 vr = gb_r[r], vi = gb_i[r];
          if constexpr (KIND == KIND_F1) {
            // pupil field P[m][n] = P0^T[n][m] * ty[m] * tx[n]  (row n, k = m)
            const f4 tr = gy_r[r] * gx_r[r] - gy_i[r] * gx_i[r];
            const f4 ti = gy_r[r] * gx_i[r] + gy_i[r] * gx_r[r];
            const f4 pr = vr * tr - vi * ti;
            const f4 pi = vr * ti + vi * tr;
            vr = pr;
            vi = pi;
          }
          fix(vr, vi, gb_k[r], a.conj_b);
          *reinterpret_cast<f4*>(&Bs[row * LDK + 4 * kq]) = vr;
          *reinterpret_cast<f4*>(&Bs[(BN + row) * LDK + 4 * kq]) = vi;
        }
      }
    };

    if (nk > 0) load_tile(k_lo);
    for (int kt = 0; kt < nk; ++kt) {
      __syncthreads();
      store_tile();
      __syncthreads();
      if (kt + 1 < nk) load_tile(k_lo + (kt + 1) * BK);

      f4 fa_r[WM], fa_i[WM], fb_r[WN], fb_i[WN];
#pragma unroll
      for (int bm = 0; bm < WM; ++bm) {
        const int r = wr * 16 * WM + bm * 16 + (lane & 15);
        fa_r[bm] = *reinterpret_cast<const f4*>(&As[r * LDK + 4 * (lane >> 4)]);
        fa_i[bm] = *reinterpret_cast<const f4*>(&As[(BM + r) * LDK + 4 * (lane >> 4)]);
      }
#pragma unroll
      for (int bn = 0; bn < WN; ++bn) {
        const int c = wc * 16 * WN + bn * 16 + (lane & 15);
        fb_r[bn] = *reinterpret_cast<const f4*>(&Bs[c * LDK + 4 * (lane >> 4)]);
        fb_i[bn] = *reinterpret_cast<const f4*>(&Bs[(BN + c) * LDK + 4 * (lane >> 4)]);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int bm = 0; bm < WM; ++bm)
#pragma unroll
          for (int bn = 0; bn < WN; ++bn) accr[bm][bn] = mfma4(fa_r[bm][s], fb_r[bn][s], accr[bm][bn]);
#pragma unroll
        for (int bm = 0; bm < WM; ++bm)
#pragma unroll
          for (int bn = 0; bn < WN; ++bn) acci[bm][bn] = mfma4(fa_r[bm][s], fb_i[bn][s], acci[bm][bn]);
#pragma unroll
        for (int bm = 0; bm < WM; ++bm) {
          const float na = -fa_i[bm][s];
#pragma unroll
          for (int bn = 0; bn < WN; ++bn) accr[bm][bn] = mfma4(na, fb_i[bn][s], accr[bm][bn]);
        }
#pragma unroll
        for (int bm = 0; bm < WM; ++bm)
#pragma unroll
          for (int bn = 0; bn < WN; ++bn) acci[bm][bn] = mfma4(fa_i[bm][s], fb_r[bn][s], acci[bm][bn]);
      }
    }

    // ------------------------------------------------------------------ per-PSF epilogue
    const int f = gb / (a.S * a.L);
    const int s = (gb / a.L) % a.S;
    const WlInfo wi = a.wl[wl];
    if constexpr (KIND == KIND_F1 || KIND == KIND_B3) {
      float* ob = a.out + (long long)lb * a.out_by_psf;
#pragma unroll
      for (int bm = 0; bm < WM; ++bm)
#pragma unroll
        for (int bn = 0; bn < WN; ++bn) {
          const int j = col0 + wc * 16 * WN + bn * 16 + (lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = row0 + wr * 16 * WM + bm * 16 + 4 * (lane >> 4) + r;
            if (i < M && j < N) {
              ob[(long long)i * a.ldo + j] = accr[bm][bn][r];
              ob[a.out_plane + (long long)i * a.ldo + j] = acci[bm][bn][r];
            }
          }
        }
    } else if constexpr (KIND == KIND_F2) {
      const float phi = a.sources[(f * a.S + s) * 3 + 2];
      const float k = wi.w * phi * wi.scale * wi.scale;
#pragma unroll
      for (int bm = 0; bm < WM; ++bm)
#pragma unroll
        for (int bn = 0; bn < WN; ++bn)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            sum[bm][bn][r] += k * (accr[bm][bn][r] * accr[bm][bn][r] + acci[bm][bn][r] * acci[bm][bn][r]);
      if (a.out) {  // keep E = c T M^T for the adjoint (fused evaluation)
        const float c = wi.scale;
        float* ob = a.out + (long long)lb * a.out_by_psf;
#pragma unroll
        for (int bm = 0; bm < WM; ++bm)
#pragma unroll
          for (int bn = 0; bn < WN; ++bn) {
            const int j = col0 + wc * 16 * WN + bn * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = row0 + wr * 16 * WM + bm * 16 + 4 * (lane >> 4) + r;
              if (i < M && j < N) {
                ob[(long long)i * a.ldo + j] = c * accr[bm][bn][r];
                ob[a.out_plane + (long long)i * a.ldo + j] = c * acci[bm][bn][r];
              }
            }
          }
      }
    } else if constexpr (KIND == KIND_B2) {
      const float phi = a.sources[(f * a.S + s) * 3 + 2];
      const float wphi = wi.w * phi;
      const float c = wi.scale;
      const int Nd = a.n_det, Q = a.Q;
      const float* rf = a.resid + (long long)f * Nd * Nd;
      float* ob = a.out + (long long)lb * a.out_by_psf;
      double part = 0.0;
#pragma unroll
      for (int bm = 0; bm < WM; ++bm)
#pragma unroll
        for (int bn = 0; bn < WN; ++bn) {
          const int j = col0 + wc * 16 * WN + bn * 16 + (lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = row0 + wr * 16 * WM + bm * 16 + 4 * (lane >> 4) + r;
            if (i < M && j < N) {
              const int p = (i / Q) * Nd + (j / Q);
              float g = a.flat[p] * rf[p];
              if (a.intrapixel) g *= a.intrapixel[(i % Q) * Q + (j % Q)];
              const float er = c * accr[bm][bn][r], ei = c * acci[bm][bn][r];
              ob[(long long)i * a.ldo + j] = wphi * g * er;
              ob[a.out_plane + (long long)i * a.ldo + j] = wphi * g * ei;
              part += (double)g * (double)(er * er + ei * ei);
            }
          }
        }
      part = wave_sum(part);
      if (lane == 0) sred[wave] = part;
      __syncthreads();
      if (tid == 0) a.red[(long long)gb * tiles + tile] = (double)wi.w * (sred[0] + sred[1] + sred[2] + sred[3]);
    } else if constexpr (KIND == KIND_B4) {
      const float c = wi.scale;
      const float kp = 2.0f * wi.kphase;
      const float* p0 = a.p0t + (long long)wl * a.p0_by_wl;
      double px = 0.0, py = 0.0;
#pragma unroll
      for (int bm = 0; bm < WM; ++bm)
#pragma unroll
        for (int bn = 0; bn < WN; ++bn) {
          const int j = col0 + wc * 16 * WN + bn * 16 + (lane & 15);       // pupil column n
          const int i0 = row0 + wr * 16 * WM + bm * 16 + 4 * (lane >> 4);  // pupil rows m = i0 .. i0+3
          if (j < N && i0 < M) {
            const f4 qr = *reinterpret_cast<const f4*>(p0 + (long long)j * a.ldp + i0);
            const f4 qi = *reinterpret_cast<const f4*>(p0 + a.p0_plane + (long long)j * a.ldp + i0);
            const f4 yr = *reinterpret_cast<const f4*>(tyb + i0);
            const f4 yi = *reinterpret_cast<const f4*>(tyb + a.tilt_plane + i0);
            const float xr = txb[j], xi = txb[a.tilt_plane + j];
            const f4 tr = yr * xr - yi * xi;
            const f4 ti = yr * xi + yi * xr;
            const f4 pr = qr * tr - qi * ti;
            const f4 pi = qr * ti + qi * tr;
            const double xj = a.xcoord[j];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = i0 + r;
              if (i < M) {
                const float g = kp * c * (pr[r] * acci[bm][bn][r] - pi[r] * accr[bm][bn][r]);
                sum[bm][bn][r] += g;
                px += xj * (double)g;
                py += a.xcoord[i] * (double)g;
              }
            }
          }
        }
      px = wave_sum(px);
      py = wave_sum(py);
      if (lane == 0) {
        sred[2 * wave] = px;
        sred[2 * wave + 1] = py;
      }
      __syncthreads();
      if (tid == 0) {
        double* o = a.red + (((long long)gb * a.ksplit + item % a.ksplit) * tiles + tile) * 2;
        o[0] = sred[0] + sred[2] + sred[4] + sred[6];
        o[1] = sred[1] + sred[3] + sred[5] + sred[7];
      }
    }
  }

  // ------------------------------------------------------------------ group epilogues
  if constexpr (KIND == KIND_F2) {
    const int Q = a.Q, Nd = a.n_det;
    __syncthreads();  // operand LDS is reused for the intensity tile
#pragma unroll
    for (int bm = 0; bm < WM; ++bm)
#pragma unroll
      for (int bn = 0; bn < WN; ++bn) {
        const int jj = wc * 16 * WN + bn * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ii = wr * 16 * WM + bm * 16 + 4 * (lane >> 4) + r;
          float v = sum[bm][bn][r];
          if (a.intrapixel) v *= a.intrapixel[(ii % Q) * Q + (jj % Q)];
          smem[ii * BN + jj] = v;
        }
      }
    __syncthreads();
    const int nbr = BM / Q, nbc = BN / Q;
    float* dst = a.part + ((long long)(a.frame0 + fl) * a.groups + grp) * Nd * Nd;
    for (int q = tid; q < nbr * nbc; q += 256) {
      const int bp = q / nbc, bq = q - bp * nbc;
      const int pr = row0 / Q + bp, pc = col0 / Q + bq;
      if (pr < Nd && pc < Nd) {
        float acc = 0.f;
        for (int u = 0; u < Q; ++u)
          for (int v = 0; v < Q; ++v) acc += smem[(bp * Q + u) * BN + bq * Q + v];
        dst[pr * Nd + pc] = acc;
      }
    }
  } else if constexpr (KIND == KIND_B4) {
    float* dst = a.part + (long long)grp * M * N;
#pragma unroll
    for (int bm = 0; bm < WM; ++bm)
#pragma unroll
      for (int bn = 0; bn < WN; ++bn) {
        const int j = col0 + wc * 16 * WN + bn * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = row0 + wr * 16 * WM + bm * 16 + 4 * (lane >> 4) + r;
          if (i < M && j < N) {
            float* d = dst + (long long)i * N + j;
            *d = (a.accumulate ? *d : 0.f) + sum[bm][bn][r];
          }
        }
      }
  }
}

template <int KIND>
hipError_t launch_kind(TileShape ts, const GemmArgs& a, int n_wg, hipStream_t st) {
  const dim3 grid(n_wg), block(256);
  if (ts.wm == 4 && ts.wn == 4) {
    hipLaunchKernelGGL((cgemm_kernel<KIND, 4, 4>), grid, block, 0, st, a);
  } else if (ts.wm == 3 && ts.wn == 3) {
    hipLaunchKernelGGL((cgemm_kernel<KIND, 3, 3>), grid, block, 0, st, a);
  } else if (ts.wm == 2 && ts.wn == 2) {
    hipLaunchKernelGGL((cgemm_kernel<KIND, 2, 2>), grid, block, 0, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

bool tile_supported(int, TileShape ts) {
  return (ts.wm == ts.wn) && (ts.wm == 4 || ts.wm == 3 || ts.wm == 2);
}

hipError_t launch_gemm(int kind, TileShape ts, const GemmArgs& a, int n_wg, hipStream_t st) {
  if (n_wg <= 0) return hipSuccess;
  switch (kind) {
    case KIND_F1: return launch_kind<KIND_F1>(ts, a, n_wg, st);
    case KIND_F2: return launch_kind<KIND_F2>(ts, a, n_wg, st);
    case KIND_B2: return launch_kind<KIND_B2>(ts, a, n_wg, st);
    case KIND_B3: return launch_kind<KIND_B3>(ts, a, n_wg, st);
    case KIND_B4: return launch_kind<KIND_B4>(ts, a, n_wg, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dlx
