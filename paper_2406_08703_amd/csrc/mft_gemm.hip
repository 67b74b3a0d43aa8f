// Batched planar-complex GEMMs of the two-sided matrix Fourier transform
// (Section 3: one product per side of the MFT) and of its adjoint, for gfx950
// on the matrix cores, in two arithmetics:
//
//   PREC 0 (DLX_FP32)   v_mfma_f32_16x16x4_f32, operands FP32, K step 16.
//   PREC 1 (DLX_BF16X3) v_mfma_f32_16x16x32_bf16, each FP32 operand x held as
//                       hi = bf16(x), lo = bf16(x - hi); a real product is
//                       hi*hi + hi*lo + lo*hi (lo*lo dropped), FP32 accumulation,
//                       K step 32. Operands arrive pre-split in HBM as four bf16
//                       planes (re hi, re lo, im hi, im lo), the same bytes as
//                       planar FP32; the operands formed in the loaders (the
//                       F1 pupil field, the B3 seed) are split at LDS store.
//
// Every stage is a "TN" product C[i][j] = sum_k A[i][k] B[j][k] with both
// operands K-contiguous, so one 128-bit LDS read per operand block feeds the
// MFMA (4 FP32 k-steps, or one 32-wide BF16 step). A workgroup of 4 waves
// (2 x 2) owns a (32 WM) x (32 WN) complex output tile; each wave holds
// WM x WN 16 x 16 blocks of real and imaginary FP32 accumulators, whose lane
// layout is the same for both instructions, so the epilogues are shared.
//
// The next K stage's global loads are issued before the MFMAs and consumed
// only when stored to LDS after them (conjugation, K-tail masking, the F1
// pupil-field product and the BF16 split happen there), so their latency
// overlaps the matrix work. The folded FP32 kernels go one step further: two
// LDS buffers, one barrier per stage, and the store of the next stage's tile
// interleaved with the current stage's MFMAs, so the loader's arithmetic and
// LDS writes issue while the matrix pipe is busy.
//
// The complex product uses the four real products Re = ArBr - AiBi,
// Im = ArBi + AiBr (no 3-multiply trick: it loses accuracy on operands of
// very different size).
//
// Stage-specific work is fused into the operand loaders (F1: P0^T times the
// row tilt; B3: the adjoint seed w phi G E from the stored field E and the
// frame's seed weights G) and into the epilogues (F1: the column tilt; F2:
// the focal-field scale; B4: the phase gradient and position sums).
//
// Two kernels implement the stages: cgemm_kernel computes the dense complex
// products, fgemm_kernel (the default) the symmetric fold of each product
// (pair sums and differences over half the depth and half the DFT rows; see
// dlx_internal.h), with the same loader and epilogue work.
#include <type_traits>

#include "dlx_internal.h"

namespace dlx {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f4 mfma_bf16(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

// RNE split of two FP32 values into packed bf16 pairs hi = bf16(x), lo = bf16(x - hi)
// (element 0 in the low half), the same rounding as split_bf16 below.
__device__ __forceinline__ void split_pair(float a, float b, unsigned int& hi, unsigned int& lo) {
  const f2 x = {a, b};
  const bf2 h = __builtin_convertvector(x, bf2);
  const f2 r = x - __builtin_convertvector(h, f2);
  hi = __builtin_bit_cast(unsigned int, h);
  lo = __builtin_bit_cast(unsigned int, __builtin_convertvector(r, bf2));
}

// RNE split of an FP32 value into bf16 hi + lo (as 16-bit patterns).
__device__ __forceinline__ void split_bf16(float x, unsigned short& hi, unsigned short& lo) {
  const __bf16 h = (__bf16)x;
  const __bf16 l = (__bf16)(x - (float)h);
  hi = __builtin_bit_cast(unsigned short, h);
  lo = __builtin_bit_cast(unsigned short, l);
}

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
// that a contiguous range of logical ids (same PSF / same wavelength, whose
// operands are shared) runs on one XCD and reuses its L2.
__device__ __forceinline__ int xcd_remap(int w, int n) {
  const int q = n >> 3, r = n & 7;
  const int xcd = w & 7, k = w >> 3;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + k;
}

// XOR swizzle of the four 16-byte k-chunks of LDS row r: a bijection on the
// chunk index for each row, and on the rows {b, b+4, b+8, b+12} and on the
// rows of one parity within 8, so that 16 consecutive rows at one chunk, or
// 4 consecutive rows at all chunks, never share a bank (32 or 64 banks).
__device__ __forceinline__ int lds_swz(int r) { return (((r >> 2) & 1) << 1) | (((r >> 1) ^ (r >> 3)) & 1); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Store one complex output element (FP32 planar, or four bf16 planes).
template <int PREC>
__device__ __forceinline__ void put(void* out, long long plane, long long idx, float re, float im) {
  if constexpr (PREC == 0) {
    float* o = static_cast<float*>(out);
    o[idx] = re;
    o[plane + idx] = im;
  } else {
    unsigned short* o = static_cast<unsigned short*>(out);
    unsigned short h, l;
    split_bf16(re, h, l);
    o[idx] = h;
    o[plane + idx] = l;
    split_bf16(im, h, l);
    o[2 * plane + idx] = h;
    o[3 * plane + idx] = l;
  }
}

template <int KIND, int WM, int WN, int PREC>
__global__ __launch_bounds__(256) void cgemm_kernel(const GemmArgs a) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  constexpr int BK = PREC == 0 ? 16 : 32;
  // LDS rows hold BK k values as four 16-byte chunks (4 FP32 or 8 bf16), unpadded; chunk kq of
  // row r sits at slot kq ^ swz(r) (see lds_swz), so the loader's stores (4 rows x 4 chunks per
  // 16 lanes) and the fragment reads (16 rows, one chunk) both spread over all LDS banks.
  constexpr int CH = PREC == 0 ? 4 : 8;
  constexpr int LDK = 4 * CH;
  constexpr int NPL = PREC == 0 ? 2 : 4;                 // planes per operand
  constexpr int A_EL = NPL * BM * LDK, B_EL = NPL * BN * LDK;
  constexpr int UNITS_A = BM * 4, UNITS_B = BN * 4;      // 16-byte k-chunks per plane row
  constexpr int A_U = (UNITS_A + 255) / 256, B_U = (UNITS_B + 255) / 256;
  using el_t = typename std::conditional<PREC == 0, float, unsigned short>::type;
  __shared__ __attribute__((aligned(16))) el_t smem[A_EL + B_EL];
  __shared__ double sred[8];
  el_t* As = smem;
  el_t* Bs = smem + A_EL;

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

  int p_begin, p_end, grp = 0;
  if constexpr (KIND == KIND_B4) {
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
    const el_t* Ab = static_cast<const el_t*>(a.A.base) + (long long)wl * a.A.by_wl + (long long)lb * a.A.by_psf;
    const float* txb = a.tx + (long long)gb * a.ldt;
    const float* tyb = a.ty + (long long)gb * a.ldt;
    // F1's B operand is the FP32 field P0^T (row tilt applied at store), B3's the FP32 field E
    // (seed applied at store); all others are el_t.
    constexpr bool kFp32B = KIND == KIND_F1 || KIND == KIND_B3;
    using bsrc_t = typename std::conditional<kFp32B, float, el_t>::type;
    // B3 with seed weights: Y = (w phi G) E formed here; without (seedw null) E already holds Y.
    float wphi = 1.f;
    const float* gwb = nullptr;
    if constexpr (KIND == KIND_B3) {
      if (a.seedw) {
        const int fs = gb / a.L;
        wphi = a.wl[wl].w * a.sources[fs * 3 + 2];
        gwb = a.seedw + (long long)(fs / a.S - a.frame0) * a.seedw_by_frame;
      }
    }
    const bsrc_t* Bb = static_cast<const bsrc_t*>(a.B.base) + (long long)wl * a.B.by_wl + (long long)lb * a.B.by_psf;

    f4 accr[WM][WN], acci[WM][WN];
#pragma unroll
    for (int bm = 0; bm < WM; ++bm)
#pragma unroll
      for (int bn = 0; bn < WN; ++bn) {
        accr[bm][bn] = f4{0.f, 0.f, 0.f, 0.f};
        acci[bm][bn] = f4{0.f, 0.f, 0.f, 0.f};
      }

    // ------------------------------------------------------------ staging registers
    // A unit = one row, 16 bytes of k per plane: 4 FP32 k (PREC 0) or 8 bf16 k (PREC 1).
    u4 ga[A_U][NPL];
    int ga_k[A_U];
    // B: el_t planes like A, except F1 which stages FP32 P0^T re/im and the row tilt,
    // and B3 which stages FP32 E re/im and the seed weight
    constexpr int BPL = (KIND == KIND_F1) ? (PREC == 0 ? 4 : 8) : (KIND == KIND_B3) ? (PREC == 0 ? 3 : 6) : NPL;
    u4 gbv[B_U][BPL];
    int gb_k[B_U];

    auto load_tile = [&](int k0) {
#pragma unroll
      for (int r = 0; r < A_U; ++r) {
        const int q = tid + 256 * r;
        const int row = q >> 2, kq = q & 3;
        const int gi = row0 + row;
        const int gk = k0 + (PREC == 0 ? 4 : 8) * kq;
        ga_k[r] = gk;
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) ga[r][pl] = u4{0u, 0u, 0u, 0u};
        if (q < UNITS_A && gi < M && gk < k_hi) {
          const el_t* p = Ab + (long long)gi * a.A.ld + gk;
#pragma unroll
          for (int pl = 0; pl < NPL; ++pl) ga[r][pl] = *reinterpret_cast<const u4*>(p + pl * a.A.plane);
        }
      }
#pragma unroll
      for (int r = 0; r < B_U; ++r) {
        const int q = tid + 256 * r;
        const int row = q >> 2, kq = q & 3;
        const int gj = col0 + row;
        const int gk = k0 + (PREC == 0 ? 4 : 8) * kq;
        gb_k[r] = gk;
#pragma unroll
        for (int pl = 0; pl < BPL; ++pl) gbv[r][pl] = u4{0u, 0u, 0u, 0u};
        if (q < UNITS_B && gj < N && gk < k_hi) {
          const bsrc_t* p = Bb + (long long)gj * a.B.ld + gk;
          if constexpr (KIND == KIND_F1) {
            // FP32 P0^T re, im and ty re, im for 4 (PREC 0) or 8 (PREC 1) consecutive k
            constexpr int V = PREC == 0 ? 1 : 2;
#pragma unroll
            for (int v = 0; v < V; ++v) {
              gbv[r][0 * V + v] = *reinterpret_cast<const u4*>(p + 4 * v);
              gbv[r][1 * V + v] = *reinterpret_cast<const u4*>(p + a.B.plane + 4 * v);
              gbv[r][2 * V + v] = *reinterpret_cast<const u4*>(tyb + gk + 4 * v);
              gbv[r][3 * V + v] = *reinterpret_cast<const u4*>(tyb + a.tilt_plane + gk + 4 * v);
            }
          } else if constexpr (KIND == KIND_B3) {
            // FP32 E re, im and G for 4 (PREC 0) or 8 (PREC 1) consecutive k
            constexpr int V = PREC == 0 ? 1 : 2;
#pragma unroll
            for (int v = 0; v < V; ++v) {
              gbv[r][0 * V + v] = *reinterpret_cast<const u4*>(p + 4 * v);
              gbv[r][1 * V + v] = *reinterpret_cast<const u4*>(p + a.B.plane + 4 * v);
              gbv[r][2 * V + v] = gwb ? *reinterpret_cast<const u4*>(gwb + (long long)gj * a.B.ld + gk + 4 * v)
                                      : __builtin_bit_cast(u4, f4{1.f, 1.f, 1.f, 1.f});
            }
          } else {
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl) gbv[r][pl] = *reinterpret_cast<const u4*>(p + pl * a.B.plane);
          }
        }
      }
    };

    // zero k >= k_hi and conjugate, on FP32 values
    auto fix32 = [&](f4& vr, f4& vi, int gk, bool conj) {
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
    // zero k >= k_hi and conjugate, on four bf16 planes of 8 k each
    auto fix16 = [&](u4* pl, int gk, bool conj) {
      if (gk + 8 > k_hi) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (gk + e >= k_hi) {
            const unsigned int mask = (e & 1) ? 0x0000ffffu : 0xffff0000u;
#pragma unroll
            for (int q = 0; q < 4; ++q) pl[q][e >> 1] &= mask;
          }
      }
      if (conj) {
        pl[2] ^= u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
        pl[3] ^= u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
      }
    };

    auto store_tile = [&]() {
#pragma unroll
      for (int r = 0; r < A_U; ++r) {
        const int q = tid + 256 * r;
        if (q < UNITS_A) {
          const int row = q >> 2, kq = q & 3;
          if constexpr (PREC == 0) {
            f4 vr = __builtin_bit_cast(f4, ga[r][0]), vi = __builtin_bit_cast(f4, ga[r][1]);
            fix32(vr, vi, ga_k[r], a.conj_a);
            *reinterpret_cast<f4*>(&As[row * LDK + 4 * (kq ^ lds_swz(row))]) = vr;
            *reinterpret_cast<f4*>(&As[(BM + row) * LDK + 4 * (kq ^ lds_swz(row))]) = vi;
          } else {
            fix16(ga[r], ga_k[r], a.conj_a);
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) *reinterpret_cast<u4*>(&As[(pl * BM + row) * LDK + 8 * (kq ^ lds_swz(row))]) = ga[r][pl];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < B_U; ++r) {
        const int q = tid + 256 * r;
        if (q < UNITS_B) {
          const int row = q >> 2, kq = q & 3;
          if constexpr (kFp32B) {
            // F1: P[m][n] / tx[n] = P0^T[n][m] * ty[m] (row n, k = m; tx is applied in the epilogue).
            // B3: Y[l][k] = (w phi G[l][k]) E[l][k].
            constexpr int V = PREC == 0 ? 1 : 2;
            f4 pr[V], pi[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
              const f4 xr = __builtin_bit_cast(f4, gbv[r][0 * V + v]), xi = __builtin_bit_cast(f4, gbv[r][1 * V + v]);
              if constexpr (KIND == KIND_F1) {
                const f4 yr = __builtin_bit_cast(f4, gbv[r][2 * V + v]), yi = __builtin_bit_cast(f4, gbv[r][3 * V + v]);
                pr[v] = xr * yr - xi * yi;
                pi[v] = xr * yi + xi * yr;
              } else {
                const f4 sw = wphi * __builtin_bit_cast(f4, gbv[r][2 * V + v]);
                pr[v] = sw * xr;
                pi[v] = sw * xi;
              }
              fix32(pr[v], pi[v], gb_k[r] + 4 * v, false);
            }
            if constexpr (PREC == 0) {
              *reinterpret_cast<f4*>(&Bs[row * LDK + 4 * (kq ^ lds_swz(row))]) = pr[0];
              *reinterpret_cast<f4*>(&Bs[(BN + row) * LDK + 4 * (kq ^ lds_swz(row))]) = pi[0];
            } else {
              unsigned int w[4][4];   // re hi, re lo, im hi, im lo: 8 k each, two per word
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int v = e >> 1, c = 2 * (e & 1);
                split_pair(pr[v][c], pr[v][c + 1], w[0][e], w[1][e]);
                split_pair(pi[v][c], pi[v][c + 1], w[2][e], w[3][e]);
              }
#pragma unroll
              for (int pl = 0; pl < 4; ++pl)
                *reinterpret_cast<u4*>(&Bs[(pl * BN + row) * LDK + 8 * (kq ^ lds_swz(row))]) =
                    u4{w[pl][0], w[pl][1], w[pl][2], w[pl][3]};
            }
          } else if constexpr (PREC == 0) {
            f4 vr = __builtin_bit_cast(f4, gbv[r][0]), vi = __builtin_bit_cast(f4, gbv[r][1]);
            fix32(vr, vi, gb_k[r], a.conj_b);
            *reinterpret_cast<f4*>(&Bs[row * LDK + 4 * (kq ^ lds_swz(row))]) = vr;
            *reinterpret_cast<f4*>(&Bs[(BN + row) * LDK + 4 * (kq ^ lds_swz(row))]) = vi;
          } else {
            fix16(gbv[r], gb_k[r], a.conj_b);
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) *reinterpret_cast<u4*>(&Bs[(pl * BN + row) * LDK + 8 * (kq ^ lds_swz(row))]) = gbv[r][pl];
          }
        }
      }
    };

    if (nk > 0) load_tile(k_lo);
    for (int kt = 0; kt < nk; ++kt) {
      __syncthreads();
      store_tile();
      __syncthreads();
      if (kt + 1 < nk) load_tile(k_lo + (kt + 1) * BK);

      if constexpr (PREC == 0) {
        f4 fa_r[WM], fa_i[WM], fb_r[WN], fb_i[WN];
#pragma unroll
        for (int bm = 0; bm < WM; ++bm) {
          const int r = wr * 16 * WM + bm * 16 + (lane & 15);
          fa_r[bm] = *reinterpret_cast<const f4*>(&As[r * LDK + 4 * ((lane >> 4) ^ lds_swz(r))]);
          fa_i[bm] = *reinterpret_cast<const f4*>(&As[(BM + r) * LDK + 4 * ((lane >> 4) ^ lds_swz(r))]);
        }
#pragma unroll
        for (int bn = 0; bn < WN; ++bn) {
          const int c = wc * 16 * WN + bn * 16 + (lane & 15);
          fb_r[bn] = *reinterpret_cast<const f4*>(&Bs[c * LDK + 4 * ((lane >> 4) ^ lds_swz(c))]);
          fb_i[bn] = *reinterpret_cast<const f4*>(&Bs[(BN + c) * LDK + 4 * ((lane >> 4) ^ lds_swz(c))]);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
          for (int bm = 0; bm < WM; ++bm)
#pragma unroll
            for (int bn = 0; bn < WN; ++bn) accr[bm][bn] = mfma_f32(fa_r[bm][s], fb_r[bn][s], accr[bm][bn]);
#pragma unroll
          for (int bm = 0; bm < WM; ++bm)
#pragma unroll
            for (int bn = 0; bn < WN; ++bn) acci[bm][bn] = mfma_f32(fa_r[bm][s], fb_i[bn][s], acci[bm][bn]);
#pragma unroll
          for (int bm = 0; bm < WM; ++bm) {
            const float na = -fa_i[bm][s];
#pragma unroll
            for (int bn = 0; bn < WN; ++bn) accr[bm][bn] = mfma_f32(na, fb_i[bn][s], accr[bm][bn]);
          }
#pragma unroll
          for (int bm = 0; bm < WM; ++bm)
#pragma unroll
            for (int bn = 0; bn < WN; ++bn) acci[bm][bn] = mfma_f32(fa_i[bm][s], fb_r[bn][s], acci[bm][bn]);
        }
      } else {
        // B fragments for all blocks, A fragments one block row at a time
        u4 fb[WN][4];
#pragma unroll
        for (int bn = 0; bn < WN; ++bn) {
          const int c = wc * 16 * WN + bn * 16 + (lane & 15);
#pragma unroll
          for (int pl = 0; pl < 4; ++pl)
            fb[bn][pl] = *reinterpret_cast<const u4*>(&Bs[(pl * BN + c) * LDK + 8 * ((lane >> 4) ^ lds_swz(c))]);
        }
#pragma unroll
        for (int bm = 0; bm < WM; ++bm) {
          const int r = wr * 16 * WM + bm * 16 + (lane & 15);
          u4 fa[4];
#pragma unroll
          for (int pl = 0; pl < 4; ++pl)
            fa[pl] = *reinterpret_cast<const u4*>(&As[(pl * BM + r) * LDK + 8 * ((lane >> 4) ^ lds_swz(r))]);
          const u4 sgn = u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
          const u4 nih = fa[2] ^ sgn, nil = fa[3] ^ sgn;   // -Ai (hi, lo)
#pragma unroll
          for (int bn = 0; bn < WN; ++bn) {
            // Re += Ar Br - Ai Bi ; Im += Ar Bi + Ai Br ; each as hi*hi + hi*lo + lo*hi
            accr[bm][bn] = mfma_bf16(fa[0], fb[bn][0], accr[bm][bn]);
            acci[bm][bn] = mfma_bf16(fa[0], fb[bn][2], acci[bm][bn]);
            accr[bm][bn] = mfma_bf16(fa[0], fb[bn][1], accr[bm][bn]);
            acci[bm][bn] = mfma_bf16(fa[0], fb[bn][3], acci[bm][bn]);
            accr[bm][bn] = mfma_bf16(fa[1], fb[bn][0], accr[bm][bn]);
            acci[bm][bn] = mfma_bf16(fa[1], fb[bn][2], acci[bm][bn]);
            accr[bm][bn] = mfma_bf16(nih, fb[bn][2], accr[bm][bn]);
            acci[bm][bn] = mfma_bf16(fa[2], fb[bn][0], acci[bm][bn]);
            accr[bm][bn] = mfma_bf16(nih, fb[bn][3], accr[bm][bn]);
            acci[bm][bn] = mfma_bf16(fa[2], fb[bn][1], acci[bm][bn]);
            accr[bm][bn] = mfma_bf16(nil, fb[bn][2], accr[bm][bn]);
            acci[bm][bn] = mfma_bf16(fa[3], fb[bn][0], acci[bm][bn]);
          }
        }
      }
    }

    // ------------------------------------------------------------------ per-PSF epilogue
    const WlInfo wi = a.wl[wl];
    if constexpr (KIND == KIND_F1 || KIND == KIND_F2 || KIND == KIND_B3) {
      // F1: T = acc * tx[n] (column tilt); F2: E = c acc, always FP32; B3: U^T = acc
      constexpr int OP = (KIND == KIND_F2) ? 0 : PREC;
      void* ob = (OP == 0) ? static_cast<void*>(static_cast<float*>(a.out) + (long long)lb * a.out_by_psf)
                           : static_cast<void*>(static_cast<unsigned short*>(a.out) + (long long)lb * a.out_by_psf);
#pragma unroll
      for (int bm = 0; bm < WM; ++bm)
#pragma unroll
        for (int bn = 0; bn < WN; ++bn) {
          const int j = col0 + wc * 16 * WN + bn * 16 + (lane & 15);
          float cr = 1.f, ci = 0.f;
          if constexpr (KIND == KIND_F1) {
            if (j < N) {
              cr = txb[j];
              ci = txb[a.tilt_plane + j];
            }
          } else if constexpr (KIND == KIND_F2) {
            cr = wi.scale;
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = row0 + wr * 16 * WM + bm * 16 + 4 * (lane >> 4) + r;
            if (i < M && j < N) {
              const float xr = accr[bm][bn][r], xi = acci[bm][bn][r];
              float re, im;
              if constexpr (KIND == KIND_F1) {
                re = xr * cr - xi * ci;
                im = xr * ci + xi * cr;
              } else {
                re = cr * xr;
                im = cr * xi;
              }
              put<OP>(ob, a.out_plane, (long long)i * a.ldo + j, re, im);
            }
          }
        }
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

  // ------------------------------------------------------------------ group epilogue
  if constexpr (KIND == KIND_B4) {
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

// ------------------------------------------------------------------------------------------------
// Folded stages (see the symmetric fold in dlx_internal.h). The DFT operand is A for F1, B3, B4
// and B for F2; it is read as in the dense kernel, restricted to the first ceil(N/2) rows and
// columns. The data operand is always FP32 in HBM: its natural chunk at k and its mirror chunk at
// ld - CH - k are loaded together, the stage's loader product is applied to each (F1: the row
// tilt ty[k] and its conjugate, which is the tilt at the mirror row; B3: w phi G), and the sum and
// difference go to LDS as four planes (Xe re, Xe im, Xo re, Xo im), split to bf16 hi/lo under
// BF16X3. Each 16 x 16 block keeps four accumulators P = (Pr, Pi), R = (Rr, Ri); the epilogue
// writes out[a] = P + i R and out[mirror a] = P - i R.
__device__ __forceinline__ f4 rev4(f4 v) { return f4{v[3], v[2], v[1], v[0]}; }

// FP32: at least two workgroups per CU. The register bound keeps B4's 64 x 64 tile at two waves
// per SIMD (its epilogue's registers would leave one); the larger FP32 shapes would spill under
// it and are not compiled (fold_tile_ok).
// The folded stage for the workgroup at logical index `lin` of its problem's own grid; `src` is the
// problem's [F][S][3] star table (read by B3 for w phi).
template <int KIND, int WM, int WN, int PREC>
__device__ __forceinline__ void fgemm_body(const GemmArgs& a, int lin, const float* src) {
  constexpr bool DA = KIND != KIND_F2;   // DFT operand on the A side (rows i), data on the B side
  constexpr int BM = 32 * WM, BN = 32 * WN;
  constexpr int BK = PREC == 0 ? 16 : 32;
  constexpr int CH = PREC == 0 ? 4 : 8;   // k per 16-byte LDS chunk
  constexpr int LDK = 4 * CH;
  constexpr int V = CH / 4;               // FP32 source vectors per chunk and plane
  constexpr int ND = PREC == 0 ? 2 : 4;   // LDS planes of the DFT operand
  constexpr int NX = PREC == 0 ? 4 : 8;   // LDS planes of the folded data operand
  constexpr int RD = DA ? BM : BN, RX = DA ? BN : BM;
  constexpr int D_EL = ND * RD * LDK, X_EL = NX * RX * LDK;
  constexpr int UNITS_D = RD * 4, UNITS_X = RX * 4;
  constexpr int D_U = (UNITS_D + 255) / 256, X_U = (UNITS_X + 255) / 256;
  using el_t = typename std::conditional<PREC == 0, float, unsigned short>::type;
  // FP32 runs a two-buffer pipeline (below); BF16X3 one LDS buffer
  constexpr bool PIPE = PREC == 0;
  constexpr int BUF_EL = D_EL + X_EL;
  __shared__ __attribute__((aligned(16))) el_t smem[(PIPE ? 2 : 1) * BUF_EL];
  constexpr int kPosSlots = KIND == KIND_B4 ? 32 : 1;
  __shared__ double spos[kPosSlots][4][2];   // B4: per-PSF, per-wave position partials

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int tiles = a.tiles_m * a.tiles_n;
  const int item = lin / tiles;
  if (item >= a.n_items) return;
  const int tile = lin - item * tiles;
  // In the adjoint products the DFT side's tile index varies fastest, so that the workgroups that read
  // one block of a PSF's data rows (E and G for B3, U^T for B4) run next to each other and share it in
  // L2. F1 and F2 keep the DFT tile fixed while the data tiles vary: F2's data rows (T) are already
  // shared by the workgroups of one row tile, and F1's (the pupil field) by every PSF of a wavelength.
  constexpr bool DFT_FAST = KIND == KIND_B3 || KIND == KIND_B4;
  const int tm = DFT_FAST ? tile % a.tiles_m : tile / a.tiles_n;
  const int tn = DFT_FAST ? tile / a.tiles_m : tile - tm * a.tiles_n;
  const int row0 = tm * BM, col0 = tn * BN;
  const int M = a.M, N = a.N, K = a.K;
  const int rowD0 = DA ? row0 : col0, rowX0 = DA ? col0 : row0;
  const int nD = DA ? M : N, nX = DA ? N : M;
  const Operand& OD = DA ? a.A : a.B;
  const Operand& OX = DA ? a.B : a.A;
  const bool conj_d = DA ? a.conj_a : a.conj_b;
  const int kmid = a.kodd ? K - 1 : -1;   // the unpaired middle term of an odd contracted length

  int p_begin, p_end, grp = 0;
  if constexpr (KIND == KIND_B4) {
    grp = item;
    const int g = item / a.ksplit;
    p_begin = g * a.group_size;
    p_end = min(p_begin + a.group_size, a.n_chunk_psf);
  } else {
    p_begin = item;
    p_end = item + 1;
  }

  f4 slo[WM][WN], shi[WM][WN];   // B4: dL/dOPD of the rows a and mirror a, summed over the group
#pragma unroll
  for (int bm = 0; bm < WM; ++bm)
#pragma unroll
    for (int bn = 0; bn < WN; ++bn) {
      slo[bm][bn] = f4{0.f, 0.f, 0.f, 0.f};
      shi[bm][bn] = f4{0.f, 0.f, 0.f, 0.f};
    }

  int k_lo = 0, k_hi = K;
  if constexpr (KIND == KIND_B4) {
    const int ks = item % a.ksplit;
    const int kc = ((K + a.ksplit * BK - 1) / (a.ksplit * BK)) * BK;
    k_lo = ks * kc;
    k_hi = min(K, k_lo + kc);
  }
  const int nk = k_hi > k_lo ? (k_hi - k_lo + BK - 1) / BK : 0;

  // Items run wavelength-major: item it is the chunk's PSF (it % nfs) L + it / nfs, so consecutive
  // items (and the contiguous workgroup ranges of one XCD) share a wavelength's DFT matrix (and, for
  // F1, its pupil field) in that XCD's L2. The PSF index itself is (frame S + star) L + wavelength.
  const int nfs = a.n_chunk_psf / a.L;
  const int ldx = OX.ld;
  // The PSF whose tiles the loader fetches: its operand bases, its row tilt (F1) and, for B3, the
  // seed weights and w phi. B4 workgroups run several PSFs; there the last k-stages of one PSF
  // already store and fetch the first tiles of the next, so a new PSF does not start on an empty
  // pipeline.
  const el_t* Db = nullptr;
  const float* Xb = nullptr;
  const float* tyl = nullptr;
  float wphi = 1.f;
  const float* gwb = nullptr;
  auto set_loader = [&](int it) {
    const int lb = (it % nfs) * a.L + it / nfs;
    const int gb = a.psf0 + lb;
    const int wl = gb % a.L;
    Db = static_cast<const el_t*>(OD.base) + (long long)wl * OD.by_wl + (long long)lb * OD.by_psf;
    Xb = static_cast<const float*>(OX.base) + (long long)wl * OX.by_wl + (long long)lb * OX.by_psf;
    tyl = a.ty + (long long)gb * a.ldt;
    if constexpr (KIND == KIND_B3) {
      if (a.seedw) {
        const int fs = gb / a.L;
        wphi = a.wl[wl].w * src[fs * 3 + 2];
        gwb = a.seedw + (long long)(fs / a.S - a.frame0) * a.seedw_by_frame;
      }
    }
  };

  // ------------------------------------------------------------ staging registers
  u4 gd[D_U][ND];
  int gd_k[D_U];
  u4 xn[X_U][2 * V], xm[X_U][2 * V];   // re, im at the natural chunk and at the mirror chunk
  u4 w0[X_U][V], w1[X_U][V];           // F1: ty re, im at k; B3: G at k and at the mirror
  int gx_k[X_U];

  auto load_tile = [&](int k0) {
#pragma unroll
    for (int r = 0; r < D_U; ++r) {
      const int q = tid + 256 * r;
      const int row = q >> 2, kq = q & 3;
      const int gi = rowD0 + row;
      const int gk = k0 + CH * kq;
      gd_k[r] = gk;
#pragma unroll
      for (int pl = 0; pl < ND; ++pl) gd[r][pl] = u4{0u, 0u, 0u, 0u};
      if (q < UNITS_D && gi < nD && gk < k_hi) {
        const el_t* p = Db + (long long)gi * OD.ld + gk;
#pragma unroll
        for (int pl = 0; pl < ND; ++pl) gd[r][pl] = *reinterpret_cast<const u4*>(p + pl * OD.plane);
      }
    }
#pragma unroll
    for (int r = 0; r < X_U; ++r) {
      const int q = tid + 256 * r;
      const int row = q >> 2, kq = q & 3;
      const int gj = rowX0 + row;
      const int gk = k0 + CH * kq;
      gx_k[r] = gk;
#pragma unroll
      for (int v = 0; v < 2 * V; ++v) {
        xn[r][v] = u4{0u, 0u, 0u, 0u};
        xm[r][v] = u4{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        w0[r][v] = u4{0u, 0u, 0u, 0u};
        w1[r][v] = u4{0u, 0u, 0u, 0u};
      }
      if (q < UNITS_X && gj < nX && gk < k_hi) {
        const float* p = Xb + (long long)gj * ldx + gk;
        const float* pm = Xb + (long long)gj * ldx + (ldx - CH - gk);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          xn[r][v] = *reinterpret_cast<const u4*>(p + 4 * v);
          xn[r][V + v] = *reinterpret_cast<const u4*>(p + OX.plane + 4 * v);
          xm[r][v] = *reinterpret_cast<const u4*>(pm + 4 * v);
          xm[r][V + v] = *reinterpret_cast<const u4*>(pm + OX.plane + 4 * v);
        }
        if constexpr (KIND == KIND_F1) {
#pragma unroll
          for (int v = 0; v < V; ++v) {
            w0[r][v] = *reinterpret_cast<const u4*>(tyl + gk + 4 * v);
            w1[r][v] = *reinterpret_cast<const u4*>(tyl + a.tilt_plane + gk + 4 * v);
          }
        } else if constexpr (KIND == KIND_B3) {
          const f4 one = f4{1.f, 1.f, 1.f, 1.f};
#pragma unroll
          for (int v = 0; v < V; ++v) {
            w0[r][v] = gwb ? *reinterpret_cast<const u4*>(gwb + (long long)gj * ldx + gk + 4 * v)
                           : __builtin_bit_cast(u4, one);
            w1[r][v] = gwb ? *reinterpret_cast<const u4*>(gwb + (long long)gj * ldx + (ldx - CH - gk) + 4 * v)
                           : __builtin_bit_cast(u4, one);
          }
        }
      }
    }
  };

  // The pipelined path's loader: every thread loads unconditionally from clamped addresses (rows
  // past the operand repeat its last row, k past k_hi its last chunk), so the loads and the stores
  // of a full tile carry no branches. Repeated rows only feed outputs that are never stored; the
  // masked store zeroes the k past k_hi, as gd_k and gx_k keep the unclamped positions.
  const int kc_last = k_hi > 0 ? ((k_hi - 1) / CH) * CH : 0;
  auto load_tile_c = [&](int k0) {
#pragma unroll
    for (int r = 0; r < D_U; ++r) {
      const int q = (tid + 256 * r) % UNITS_D;
      const int row = q >> 2, kq = q & 3;
      const int gi = min(rowD0 + row, nD - 1);
      const int gk = k0 + CH * kq;
      gd_k[r] = gk;
      const el_t* p = Db + (long long)gi * OD.ld + min(gk, kc_last);
#pragma unroll
      for (int pl = 0; pl < ND; ++pl) gd[r][pl] = *reinterpret_cast<const u4*>(p + pl * OD.plane);
    }
#pragma unroll
    for (int r = 0; r < X_U; ++r) {
      const int q = (tid + 256 * r) % UNITS_X;
      const int row = q >> 2, kq = q & 3;
      const int gj = min(rowX0 + row, nX - 1);
      const int gk = k0 + CH * kq;
      const int gkc = min(gk, kc_last);
      gx_k[r] = gk;
      const float* p = Xb + (long long)gj * ldx + gkc;
      const float* pm = Xb + (long long)gj * ldx + (ldx - CH - gkc);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        xn[r][v] = *reinterpret_cast<const u4*>(p + 4 * v);
        xn[r][V + v] = *reinterpret_cast<const u4*>(p + OX.plane + 4 * v);
        xm[r][v] = *reinterpret_cast<const u4*>(pm + 4 * v);
        xm[r][V + v] = *reinterpret_cast<const u4*>(pm + OX.plane + 4 * v);
      }
      if constexpr (KIND == KIND_F1) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          w0[r][v] = *reinterpret_cast<const u4*>(tyl + gkc + 4 * v);
          w1[r][v] = *reinterpret_cast<const u4*>(tyl + a.tilt_plane + gkc + 4 * v);
        }
      } else if constexpr (KIND == KIND_B3) {
        // without seed weights (the seed pass) G is 1: the data rows stand in as a valid address
        const bool hg = gwb != nullptr;
        const float* g = hg ? gwb : Xb;
        const u4 one = __builtin_bit_cast(u4, f4{1.f, 1.f, 1.f, 1.f});
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const u4 g0 = *reinterpret_cast<const u4*>(g + (long long)gj * ldx + gkc + 4 * v);
          const u4 g1 = *reinterpret_cast<const u4*>(g + (long long)gj * ldx + (ldx - CH - gkc) + 4 * v);
          w0[r][v] = hg ? g0 : one;
          w1[r][v] = hg ? g1 : one;
        }
      }
    }
  };

  // Staged tile -> LDS buffer `buf`. MASK: zero the K tail and the unpaired middle term (a tile
  // that reaches k_hi or kmid); without it the tile must lie wholly inside both. The pipelined path
  // leaves the DFT operand unconjugated and negates the accumulators that take its imaginary part.
  auto store_tile = [&](el_t* buf, auto mask_tag) {
    // the loader products are rounded before the pair sums (no FMA contraction), as a separately
    // formed seed or the dense kernel's loader would round them, whatever the masking
#pragma clang fp contract(off)
    constexpr bool MASK = decltype(mask_tag)::value;
    el_t* Ds = buf;
    el_t* Xs = buf + D_EL;
    // DFT operand: as the dense kernel (K tail masked, conjugated for the adjoint)
#pragma unroll
    for (int r = 0; r < D_U; ++r) {
      // the pipelined loader gives threads past the tile's units a copy of a unit (q mod units):
      // they store the same words to the same place, so no thread branches off
      const int q = PIPE ? (tid + 256 * r) % UNITS_D : tid + 256 * r;
      if (PIPE || UNITS_D % 256 == 0 || q < UNITS_D) {
        const int row = q >> 2, kq = q & 3;
        if constexpr (PREC == 0) {
          f4 vr = __builtin_bit_cast(f4, gd[r][0]), vi = __builtin_bit_cast(f4, gd[r][1]);
          const int gk = gd_k[r];
          if (MASK && gk + 4 > k_hi) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (gk + e >= k_hi) {
                vr[e] = 0.f;
                vi[e] = 0.f;
              }
          }
          if (!PIPE && conj_d) vi = -vi;
          *reinterpret_cast<f4*>(&Ds[row * LDK + 4 * (kq ^ lds_swz(row))]) = vr;
          *reinterpret_cast<f4*>(&Ds[(RD + row) * LDK + 4 * (kq ^ lds_swz(row))]) = vi;
        } else {
          u4* pl = gd[r];
          const int gk = gd_k[r];
          if (MASK && gk + 8 > k_hi) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if (gk + e >= k_hi) {
                const unsigned int mask = (e & 1) ? 0x0000ffffu : 0xffff0000u;
#pragma unroll
                for (int c = 0; c < 4; ++c) pl[c][e >> 1] &= mask;
              }
          }
          if (conj_d) {
            pl[2] ^= u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
            pl[3] ^= u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
          }
#pragma unroll
          for (int c = 0; c < 4; ++c)
            *reinterpret_cast<u4*>(&Ds[(c * RD + row) * LDK + 8 * (kq ^ lds_swz(row))]) = pl[c];
        }
      }
    }
    // data operand: loader product at k and at the mirror, then sum and difference
#pragma unroll
    for (int r = 0; r < X_U; ++r) {
      const int q = PIPE ? (tid + 256 * r) % UNITS_X : tid + 256 * r;
      if (PIPE || UNITS_X % 256 == 0 || q < UNITS_X) {
        const int row = q >> 2, kq = q & 3;
        f4 er[V], ei[V], odr[V], odi[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          f4 xr = __builtin_bit_cast(f4, xn[r][v]), xi = __builtin_bit_cast(f4, xn[r][V + v]);
          // the mirror of natural element 4v + e is element 3 - e of mirror vector V - 1 - v
          f4 yr = rev4(__builtin_bit_cast(f4, xm[r][V - 1 - v]));
          f4 yi = rev4(__builtin_bit_cast(f4, xm[r][2 * V - 1 - v]));
          if constexpr (KIND == KIND_F1) {
            // P[k] = P0[k] ty[k]; at the mirror row the tilt is conj(ty[k])
            const f4 tr = __builtin_bit_cast(f4, w0[r][v]), ti = __builtin_bit_cast(f4, w1[r][v]);
            const f4 ar = xr * tr - xi * ti, ai = xr * ti + xi * tr;
            const f4 br = yr * tr + yi * ti, bi = yi * tr - yr * ti;
            xr = ar;
            xi = ai;
            yr = br;
            yi = bi;
          } else if constexpr (KIND == KIND_B3) {
            const f4 g = wphi * __builtin_bit_cast(f4, w0[r][v]);
            const f4 gm = wphi * rev4(__builtin_bit_cast(f4, w1[r][V - 1 - v]));
            xr = g * xr;
            xi = g * xi;
            yr = gm * yr;
            yi = gm * yi;
          }
          // K tail and the unpaired middle term (assigned after the products: padding is not read)
          const int kb = gx_k[r] + 4 * v;
          if (MASK && (kb + 4 > k_hi || (kmid >= kb && kmid < kb + 4))) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              if (kb + e >= k_hi) {
                xr[e] = 0.f;
                xi[e] = 0.f;
                yr[e] = 0.f;
                yi[e] = 0.f;
              }
              if (kb + e == kmid) {
                yr[e] = 0.f;
                yi[e] = 0.f;
              }
            }
          }
          er[v] = xr + yr;
          ei[v] = xi + yi;
          odr[v] = xr - yr;
          odi[v] = xi - yi;
        }
        if constexpr (PREC == 0) {
          const int o = 4 * (kq ^ lds_swz(row));
          *reinterpret_cast<f4*>(&Xs[(0 * RX + row) * LDK + o]) = er[0];
          *reinterpret_cast<f4*>(&Xs[(1 * RX + row) * LDK + o]) = ei[0];
          *reinterpret_cast<f4*>(&Xs[(2 * RX + row) * LDK + o]) = odr[0];
          *reinterpret_cast<f4*>(&Xs[(3 * RX + row) * LDK + o]) = odi[0];
        } else {
          // planes: Xe re hi, lo; Xe im hi, lo; Xo re hi, lo; Xo im hi, lo (8 k each, two per word)
          unsigned int w[8][4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int v = e >> 1, c = 2 * (e & 1);
            split_pair(er[v][c], er[v][c + 1], w[0][e], w[1][e]);
            split_pair(ei[v][c], ei[v][c + 1], w[2][e], w[3][e]);
            split_pair(odr[v][c], odr[v][c + 1], w[4][e], w[5][e]);
            split_pair(odi[v][c], odi[v][c + 1], w[6][e], w[7][e]);
          }
          const int o = 8 * (kq ^ lds_swz(row));
#pragma unroll
          for (int pl = 0; pl < 8; ++pl)
            *reinterpret_cast<u4*>(&Xs[(pl * RX + row) * LDK + o]) = u4{w[pl][0], w[pl][1], w[pl][2], w[pl][3]};
        }
      }
    }
  };

  // Instruction interleave of one pipelined k-stage. F1 and B3 (sched_group_barrier masks: 0x008
  // MFMA, 0x002 VALU, 0x100 LDS read, 0x200 LDS write, 0x020 global read): the fragment reads, a
  // quarter of the MFMAs alone while they arrive, then each MFMA followed by a little of the
  // store's VALU work and LDS writes, then by the next stage's global loads. F2 and B4 take the
  // compiler's own interleave for small GEMMs (iglp_opt 1), which measured faster for them; for
  // B4 the groups above are not honoured by the scheduler at all.
  auto pipe_schedule = [&]() {
    if constexpr (PIPE && (KIND == KIND_F2 || KIND == KIND_B4)) {
      __builtin_amdgcn_iglp_opt(1);
    } else if constexpr (PIPE) {
      constexpr int WD = DA ? WM : WN, WX = DA ? WN : WM;
      constexpr int NMF = WM * WN * 16;
      constexpr int NDSR = 2 * WD + 4 * WX;
      constexpr int NDSW = 2 * D_U + 4 * X_U;
      constexpr int NVM = 2 * D_U + (KIND == KIND_F1 || KIND == KIND_B3 ? 6 : 4) * X_U;
      // B3 (the loader with the most VALU work) starts its store after two MFMAs
      constexpr int Q1 = KIND == KIND_B3 ? 2 : NMF / 4;
      constexpr int Q2 = KIND == KIND_B3 ? NMF * 3 / 4 - 2 : NMF / 2;
      constexpr int Q3 = NMF - Q1 - Q2;
      constexpr int DSW_EVERY = Q2 / NDSW;   // MFMAs per LDS write in the middle half
      static_assert(DSW_EVERY >= 1, "every LDS write needs a slot in the middle half");
      __builtin_amdgcn_sched_group_barrier(0x100, NDSR, 0);
#pragma unroll
      for (int i = 0; i < Q1; ++i) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
#pragma unroll
      for (int i = 0; i < Q2; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
        if (i % DSW_EVERY == DSW_EVERY - 1) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
      }
#pragma unroll
      for (int i = 0; i < Q3; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);
        if (i < NVM) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
      }
    }
  };

  // pipelined stream state: the tile count, the PSF the loader points at, the full k-stages
  int ts = 0, lpsf = p_begin;
  const int k_full = a.kodd ? min(k_hi, K - 1) : k_hi;
  const int nfull = max(0, (k_full - k_lo) / BK);   // k-stages [0, nfull) hold full tiles
  for (int it = p_begin; it < p_end; ++it) {
    const int lb = (it % nfs) * a.L + it / nfs;
    const int gb = a.psf0 + lb;
    const int wl = gb % a.L;
    const float* txb = a.tx + (long long)gb * a.ldt;
    const float* tyb = a.ty + (long long)gb * a.ldt;

    f4 pr_[WM][WN], pi_[WM][WN], rr_[WM][WN], ri_[WM][WN];
#pragma unroll
    for (int bm = 0; bm < WM; ++bm)
#pragma unroll
      for (int bn = 0; bn < WN; ++bn) {
        pr_[bm][bn] = f4{0.f, 0.f, 0.f, 0.f};
        pi_[bm][bn] = f4{0.f, 0.f, 0.f, 0.f};
        rr_[bm][bn] = f4{0.f, 0.f, 0.f, 0.f};
        ri_[bm][bn] = f4{0.f, 0.f, 0.f, 0.f};
      }
    // the matrix work of one k-stage, from the operands in LDS buffer `buf`
    auto mma = [&](const el_t* buf) {
      const el_t* Ds = buf;
      const el_t* Xs = buf + D_EL;
      if constexpr (PREC == 0) {
        constexpr int WD = DA ? WM : WN, WX = DA ? WN : WM;
        const int bd = DA ? wr : wc, bx = DA ? wc : wr;
        f4 dr[WD], di[WD], xf[WX][4];
#pragma unroll
        for (int b = 0; b < WD; ++b) {
          const int r = bd * 16 * WD + b * 16 + (lane & 15);
          const int o = 4 * ((lane >> 4) ^ lds_swz(r));
          dr[b] = *reinterpret_cast<const f4*>(&Ds[r * LDK + o]);
          di[b] = *reinterpret_cast<const f4*>(&Ds[(RD + r) * LDK + o]);
        }
#pragma unroll
        for (int b = 0; b < WX; ++b) {
          const int r = bx * 16 * WX + b * 16 + (lane & 15);
          const int o = 4 * ((lane >> 4) ^ lds_swz(r));
#pragma unroll
          for (int pl = 0; pl < 4; ++pl) xf[b][pl] = *reinterpret_cast<const f4*>(&Xs[(pl * RX + r) * LDK + o]);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
          for (int bm = 0; bm < WM; ++bm)
#pragma unroll
            for (int bn = 0; bn < WN; ++bn) {
              const int id = DA ? bm : bn, ix = DA ? bn : bm;
              if constexpr (DA) {
                pr_[bm][bn] = mfma_f32(dr[id][s], xf[ix][0][s], pr_[bm][bn]);
                pi_[bm][bn] = mfma_f32(dr[id][s], xf[ix][1][s], pi_[bm][bn]);
                rr_[bm][bn] = mfma_f32(di[id][s], xf[ix][2][s], rr_[bm][bn]);
                ri_[bm][bn] = mfma_f32(di[id][s], xf[ix][3][s], ri_[bm][bn]);
              } else {
                pr_[bm][bn] = mfma_f32(xf[ix][0][s], dr[id][s], pr_[bm][bn]);
                pi_[bm][bn] = mfma_f32(xf[ix][1][s], dr[id][s], pi_[bm][bn]);
                rr_[bm][bn] = mfma_f32(xf[ix][2][s], di[id][s], rr_[bm][bn]);
                ri_[bm][bn] = mfma_f32(xf[ix][3][s], di[id][s], ri_[bm][bn]);
              }
            }
        }
      } else {
        // each real product as hi*hi + hi*lo + lo*hi
        if constexpr (DA) {
          u4 xf[WN][8];
#pragma unroll
          for (int bn = 0; bn < WN; ++bn) {
            const int c = wc * 16 * WN + bn * 16 + (lane & 15);
            const int o = 8 * ((lane >> 4) ^ lds_swz(c));
#pragma unroll
            for (int pl = 0; pl < 8; ++pl) xf[bn][pl] = *reinterpret_cast<const u4*>(&Xs[(pl * RX + c) * LDK + o]);
          }
#pragma unroll
          for (int bm = 0; bm < WM; ++bm) {
            const int r = wr * 16 * WM + bm * 16 + (lane & 15);
            const int o = 8 * ((lane >> 4) ^ lds_swz(r));
            u4 d[4];
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) d[pl] = *reinterpret_cast<const u4*>(&Ds[(pl * RD + r) * LDK + o]);
#pragma unroll
            for (int bn = 0; bn < WN; ++bn) {
              pr_[bm][bn] = mfma_bf16(d[0], xf[bn][0], pr_[bm][bn]);
              pi_[bm][bn] = mfma_bf16(d[0], xf[bn][2], pi_[bm][bn]);
              rr_[bm][bn] = mfma_bf16(d[2], xf[bn][4], rr_[bm][bn]);
              ri_[bm][bn] = mfma_bf16(d[2], xf[bn][6], ri_[bm][bn]);
              pr_[bm][bn] = mfma_bf16(d[0], xf[bn][1], pr_[bm][bn]);
              pi_[bm][bn] = mfma_bf16(d[0], xf[bn][3], pi_[bm][bn]);
              rr_[bm][bn] = mfma_bf16(d[2], xf[bn][5], rr_[bm][bn]);
              ri_[bm][bn] = mfma_bf16(d[2], xf[bn][7], ri_[bm][bn]);
              pr_[bm][bn] = mfma_bf16(d[1], xf[bn][0], pr_[bm][bn]);
              pi_[bm][bn] = mfma_bf16(d[1], xf[bn][2], pi_[bm][bn]);
              rr_[bm][bn] = mfma_bf16(d[3], xf[bn][4], rr_[bm][bn]);
              ri_[bm][bn] = mfma_bf16(d[3], xf[bn][6], ri_[bm][bn]);
            }
          }
        } else {
          u4 d[WN][4];
#pragma unroll
          for (int bn = 0; bn < WN; ++bn) {
            const int c = wc * 16 * WN + bn * 16 + (lane & 15);
            const int o = 8 * ((lane >> 4) ^ lds_swz(c));
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) d[bn][pl] = *reinterpret_cast<const u4*>(&Ds[(pl * RD + c) * LDK + o]);
          }
#pragma unroll
          for (int bm = 0; bm < WM; ++bm) {
            const int r = wr * 16 * WM + bm * 16 + (lane & 15);
            const int o = 8 * ((lane >> 4) ^ lds_swz(r));
            u4 x[8];
#pragma unroll
            for (int pl = 0; pl < 8; ++pl) x[pl] = *reinterpret_cast<const u4*>(&Xs[(pl * RX + r) * LDK + o]);
#pragma unroll
            for (int bn = 0; bn < WN; ++bn) {
              pr_[bm][bn] = mfma_bf16(x[0], d[bn][0], pr_[bm][bn]);
              pi_[bm][bn] = mfma_bf16(x[2], d[bn][0], pi_[bm][bn]);
              rr_[bm][bn] = mfma_bf16(x[4], d[bn][2], rr_[bm][bn]);
              ri_[bm][bn] = mfma_bf16(x[6], d[bn][2], ri_[bm][bn]);
              pr_[bm][bn] = mfma_bf16(x[0], d[bn][1], pr_[bm][bn]);
              pi_[bm][bn] = mfma_bf16(x[2], d[bn][1], pi_[bm][bn]);
              rr_[bm][bn] = mfma_bf16(x[4], d[bn][3], rr_[bm][bn]);
              ri_[bm][bn] = mfma_bf16(x[6], d[bn][3], ri_[bm][bn]);
              pr_[bm][bn] = mfma_bf16(x[1], d[bn][0], pr_[bm][bn]);
              pi_[bm][bn] = mfma_bf16(x[3], d[bn][0], pi_[bm][bn]);
              rr_[bm][bn] = mfma_bf16(x[5], d[bn][2], rr_[bm][bn]);
              ri_[bm][bn] = mfma_bf16(x[7], d[bn][2], ri_[bm][bn]);
            }
          }
        }
      }
    };

    if constexpr (!PIPE) {
      if (KIND != KIND_B4 || it == p_begin) {   // later B4 PSFs were fetched by the previous PSF
        set_loader(it);
        if (nk > 0) load_tile(k_lo);
      }
      for (int kt = 0; kt < nk; ++kt) {
        __syncthreads();
        store_tile(smem, std::true_type{});
        __syncthreads();
        if (kt + 1 < nk) {
          load_tile(k_lo + (kt + 1) * BK);
        } else if (KIND == KIND_B4 && it + 1 < p_end) {
          set_loader(it + 1);
          load_tile(k_lo);
        }
        mma(smem);
      }
    } else if constexpr (KIND != KIND_B4) {
      // Two LDS buffers and one barrier per k-stage: the MFMAs of stage kt read buffer kt & 1 while
      // the tile of stage kt + 1, staged in registers, is stored into the other buffer and the
      // loads of stage kt + 2 go out. For full tiles the store is branch-free and the scheduler
      // is told to spread it, and the loads, between the MFMAs, so the pair sums and the LDS and
      // global traffic issue while the matrix pipe is busy. (One workgroup runs one PSF here.)
      set_loader(it);
      load_tile_c(k_lo);
      if (nfull > 0)
        store_tile(smem, std::false_type{});
      else
        store_tile(smem, std::true_type{});
      load_tile_c(k_lo + BK);
      __syncthreads();
      int kt = 0;
      for (; kt + 1 < nfull; ++kt) {   // the next tile is full: one basic block per stage
        mma(smem + (kt & 1) * BUF_EL);
        store_tile(smem + ((kt + 1) & 1) * BUF_EL, std::false_type{});
        load_tile_c(k_lo + (kt + 2) * BK);
        pipe_schedule();
        __syncthreads();
      }
      for (; kt < nk; ++kt) {   // the last one or two stages
        mma(smem + (kt & 1) * BUF_EL);
        if (kt + 1 < nk) {
          store_tile(smem + ((kt + 1) & 1) * BUF_EL, std::true_type{});
          load_tile_c(k_lo + (kt + 2) * BK);
        }
        __syncthreads();
      }
    } else if (nk > 0) {
      // B4: the same pipeline over a stream of tiles that runs through the workgroup's PSFs and
      // their k-stages (tile ts in buffer ts & 1), so the first tiles of a PSF are stored and
      // fetched during the previous PSF's last stages.
      if (it == p_begin) {   // prologue: tile 0 to LDS, tile 1 to registers
        set_loader(it);
        lpsf = it;
        load_tile_c(k_lo);
        if (nfull > 0)
          store_tile(smem, std::false_type{});
        else
          store_tile(smem, std::true_type{});
        if (nk > 1) {
          load_tile_c(k_lo + BK);
        } else if (it + 1 < p_end) {
          set_loader(it + 1);
          lpsf = it + 1;
          load_tile_c(k_lo);
        }
        __syncthreads();
      }
      const int nfast = min(nfull - 1, nk - 2);   // next tile full, the tile after in this PSF
      int kt = 0;
      for (; kt < nfast; ++kt, ++ts) {   // one basic block per stage
        mma(smem + (ts & 1) * BUF_EL);
        store_tile(smem + ((ts + 1) & 1) * BUF_EL, std::false_type{});
        load_tile_c(k_lo + (kt + 2) * BK);
        pipe_schedule();
        __syncthreads();
      }
      for (; kt < nk; ++kt, ++ts) {   // the PSF's last stages, with masking and the PSF switch
        mma(smem + (ts & 1) * BUF_EL);
        if (kt + 1 < nk || it + 1 < p_end) store_tile(smem + ((ts + 1) & 1) * BUF_EL, std::true_type{});
        int lk = kt + 2, lp = it;   // the tile two ahead in the stream
        while (lk >= nk) {
          lk -= nk;
          ++lp;
        }
        if (lp < p_end) {
          if (lp != lpsf) {
            set_loader(lp);
            lpsf = lp;
          }
          load_tile_c(k_lo + lk * BK);
        }
        __syncthreads();
      }
    }
    if constexpr (PIPE) {
      if (conj_d) {   // the adjoint's conj(M): its imaginary part feeds R only
#pragma unroll
        for (int bm = 0; bm < WM; ++bm)
#pragma unroll
          for (int bn = 0; bn < WN; ++bn) {
            rr_[bm][bn] = -rr_[bm][bn];
            ri_[bm][bn] = -ri_[bm][bn];
          }
      }
    }

    // ------------------------------------------------------------------ per-PSF epilogue
    // out[a] = P + i R = (Pr - Ri, Pi + Rr);  out[mirror a] = P - i R = (Pr + Ri, Pi - Rr)
    const WlInfo wi = a.wl[wl];
    if constexpr (KIND == KIND_F1 || KIND == KIND_F2 || KIND == KIND_B3) {
      float* ob = static_cast<float*>(a.out) + (long long)lb * a.out_by_psf;
#pragma unroll
      for (int bm = 0; bm < WM; ++bm)
#pragma unroll
        for (int bn = 0; bn < WN; ++bn) {
          const int j = col0 + wc * 16 * WN + bn * 16 + (lane & 15);
          float cr = 1.f, ci = 0.f;
          if constexpr (KIND == KIND_F1) {
            if (j < N) {
              cr = txb[j];
              ci = txb[a.tilt_plane + j];
            }
          } else if constexpr (KIND == KIND_F2) {
            cr = wi.scale;
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = row0 + wr * 16 * WM + bm * 16 + 4 * (lane >> 4) + r;
            if (i < M && j < N) {
              const float Pr = pr_[bm][bn][r], Pi = pi_[bm][bn][r], Rr = rr_[bm][bn][r], Ri = ri_[bm][bn][r];
              const float lr = Pr - Ri, li = Pi + Rr, hr = Pr + Ri, hi = Pi - Rr;
              if constexpr (KIND == KIND_F2) {
                // mirrored index: the output column
                const int jm = a.mirror_n - 1 - j;
                const long long base = (long long)i * a.ldo;
                const long long i0 = base + (j < a.out_h ? j : j + a.out_s);
                ob[i0] = cr * lr;
                ob[a.out_plane + i0] = cr * li;
                if (jm != j) {
                  const long long i1 = base + (jm < a.out_h ? jm : jm + a.out_s);
                  ob[i1] = cr * hr;
                  ob[a.out_plane + i1] = cr * hi;
                }
              } else {
                // mirrored index: the output row
                const int im = a.mirror_n - 1 - i;
                const int jc = j < a.out_h ? j : j + a.out_s;
                float ar = lr, ai = li, br = hr, bi = hi;
                if constexpr (KIND == KIND_F1) {   // column tilt tx[n]
                  ar = lr * cr - li * ci;
                  ai = lr * ci + li * cr;
                  br = hr * cr - hi * ci;
                  bi = hr * ci + hi * cr;
                }
                const long long i0 = (long long)i * a.ldo + jc;
                ob[i0] = ar;
                ob[a.out_plane + i0] = ai;
                if (im != i) {
                  const long long i1 = (long long)im * a.ldo + jc;
                  ob[i1] = br;
                  ob[a.out_plane + i1] = bi;
                }
              }
            }
          }
        }
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
          const int i0 = row0 + wr * 16 * WM + bm * 16 + 4 * (lane >> 4);  // pupil rows m = i0 .. i0+3 (< ceil(Ni/2))
          if (j < N && i0 < M) {
            // P0^T at rows m and at their mirrors Ni-1-m (stored at ld-1-m), the tilts
            const float* q = p0 + (long long)j * a.ldp;
            const f4 qr = *reinterpret_cast<const f4*>(q + i0);
            const f4 qi = *reinterpret_cast<const f4*>(q + a.p0_plane + i0);
            const f4 mr = rev4(*reinterpret_cast<const f4*>(q + (a.ldp - 4 - i0)));
            const f4 mi = rev4(*reinterpret_cast<const f4*>(q + a.p0_plane + (a.ldp - 4 - i0)));
            const f4 yr = *reinterpret_cast<const f4*>(tyb + i0);
            const f4 yi = *reinterpret_cast<const f4*>(tyb + a.tilt_plane + i0);
            const float xr = txb[j], xi = txb[a.tilt_plane + j];
            const f4 tr = yr * xr - yi * xi, ti = yr * xi + yi * xr;   // ty[m] tx[n]
            const f4 ur = yr * xr + yi * xi, ui = yr * xi - yi * xr;   // conj(ty[m]) tx[n]
            const f4 plr = qr * tr - qi * ti, pli = qr * ti + qi * tr;
            const f4 phr = mr * ur - mi * ui, phi = mr * ui + mi * ur;
            const double xj = a.xcoord[j];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = i0 + r;
              if (i < M) {
                const float Pr = pr_[bm][bn][r], Pi = pi_[bm][bn][r], Rr = rr_[bm][bn][r], Ri = ri_[bm][bn][r];
                const float g = kp * c * (plr[r] * (Pi + Rr) - pli[r] * (Pr - Ri));
                const int im = a.mirror_n - 1 - i;
                const float gm = im != i ? kp * c * (phr[r] * (Pi - Rr) - phi[r] * (Pr + Ri)) : 0.f;
                slo[bm][bn][r] += g;
                shi[bm][bn][r] += gm;
                px += xj * ((double)g + (double)gm);
                py += a.xcoord[i] * (double)g + a.xcoord[im] * (double)gm;
              }
            }
          }
        }
      px = wave_sum(px);
      py = wave_sum(py);
      // the PSF's wave sums wait in an LDS slot; they are added (in wave order) and written when
      // the slots are full or the group ends, so the workgroup does not synchronise after each PSF
      const int slot = (it - p_begin) % kPosSlots;
      if (lane == 0) {
        spos[slot][wave][0] = px;
        spos[slot][wave][1] = py;
      }
      if (slot == kPosSlots - 1 || it + 1 == p_end) {
        __syncthreads();
        if (tid <= slot) {
          const int is = it - slot + tid;
          const int gbs = a.psf0 + (is % nfs) * a.L + is / nfs;
          double* o = a.red + (((long long)gbs * a.ksplit + item % a.ksplit) * tiles + tile) * 2;
          o[0] = spos[tid][0][0] + spos[tid][1][0] + spos[tid][2][0] + spos[tid][3][0];
          o[1] = spos[tid][0][1] + spos[tid][1][1] + spos[tid][2][1] + spos[tid][3][1];
        }
        if (it + 1 < p_end) __syncthreads();   // the next PSFs reuse the slots
      }
    }
  }

  // ------------------------------------------------------------------ group epilogue
  if constexpr (KIND == KIND_B4) {
    float* dst = a.part + (long long)grp * a.mirror_n * N;
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
            *d = (a.accumulate ? *d : 0.f) + slo[bm][bn][r];
            const int im = a.mirror_n - 1 - i;
            if (im != i) {
              float* d2 = dst + (long long)im * N + j;
              *d2 = (a.accumulate ? *d2 : 0.f) + shi[bm][bn][r];
            }
          }
        }
      }
  }
}

template <int KIND, int WM, int WN, int PREC>
__global__ __launch_bounds__(256, PREC == 0 ? 2 : 1) void fgemm_kernel(const GemmArgs a) {
  fgemm_body<KIND, WM, WN, PREC>(a, xcd_remap(blockIdx.x, gridDim.x), a.sources);
}

// One launch of a folded stage over the problems of a multi-problem plan: workgroup g runs logical
// workgroup tab[g].y of problem tab[g].x, whose arguments are args[tab[g].x]; the problem's star
// table is sources + args[k].src_off (sources: the call's packed table). The table is already in
// dispatch order (the host lays it out as one queue per XCD), so no remap is applied here.
template <int KIND, int WM, int WN, int PREC>
__global__ __launch_bounds__(256, PREC == 0 ? 2 : 1) void fgemm_group_kernel(const GemmArgs* __restrict__ args,
                                                                            const int2* __restrict__ tab,
                                                                            const float* sources) {
  const int2 e = tab[blockIdx.x];
  const GemmArgs& a = args[e.x];
  fgemm_body<KIND, WM, WN, PREC>(a, e.y, sources ? sources + a.src_off : nullptr);
}

// Folded tile shapes compiled: those that keep their accumulators in registers. FP32 (two
// workgroups per CU): up to four 32 x 32 blocks, except B4's 128 x 32 and 32 x 128. BF16X3: all
// but 128 x 128 (and B4's 96 x 96 and 64 x 128, whose epilogue and prefetched next tile spill).
constexpr bool fold_tile_ok(int kind, int prec, int wm, int wn) {
  if (prec == 0) return wm * wn <= 4 && !(kind == KIND_B4 && wm != wn && wm * wn == 4);
  return !(wm == 4 && wn == 4) && !(kind == KIND_B4 && ((wm == 3 && wn == 3) || (wm == 2 && wn == 4)));
}

template <int KIND, int WM, int WN, int PREC>
hipError_t launch_fold(dim3 grid, dim3 block, const GemmArgs& a, hipStream_t st) {
  if constexpr (fold_tile_ok(KIND, PREC, WM, WN)) {
    hipLaunchKernelGGL((fgemm_kernel<KIND, WM, WN, PREC>), grid, block, 0, st, a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int KIND, int PREC>
hipError_t launch_kind(TileShape ts, const GemmArgs& a, int n_wg, hipStream_t st) {
  const dim3 grid(n_wg), block(256);
#define DLX_TILE(WM_, WN_)                                                                     \
  if (ts.wm == WM_ && ts.wn == WN_) {                                                          \
    if (a.fold) return launch_fold<KIND, WM_, WN_, PREC>(grid, block, a, st);                \
    hipLaunchKernelGGL((cgemm_kernel<KIND, WM_, WN_, PREC>), grid, block, 0, st, a);          \
    return hipGetLastError();                                                                  \
  }
  DLX_TILE(4, 4)
  DLX_TILE(3, 3)
  DLX_TILE(2, 2)
  DLX_TILE(4, 2)
  DLX_TILE(2, 4)
  DLX_TILE(2, 1)
  DLX_TILE(1, 2)
  DLX_TILE(1, 1)
  DLX_TILE(4, 1)
  DLX_TILE(1, 4)
#undef DLX_TILE
  return hipErrorInvalidValue;
}

template <int PREC>
hipError_t launch_prec(int kind, TileShape ts, const GemmArgs& a, int n_wg, hipStream_t st) {
  switch (kind) {
    case KIND_F1: return launch_kind<KIND_F1, PREC>(ts, a, n_wg, st);
    case KIND_F2: return launch_kind<KIND_F2, PREC>(ts, a, n_wg, st);
    case KIND_B3: return launch_kind<KIND_B3, PREC>(ts, a, n_wg, st);
    case KIND_B4: return launch_kind<KIND_B4, PREC>(ts, a, n_wg, st);
    default: return hipErrorInvalidValue;
  }
}

template <int KIND, int PREC>
hipError_t launch_group_kind(TileShape ts, const GemmArgs* args, const int2* tab, int n_wg, const float* sources,
                             hipStream_t st) {
  const dim3 grid(n_wg), block(256);
#define DLX_TILE(WM_, WN_)                                                                                   \
  if (ts.wm == WM_ && ts.wn == WN_) {                                                                        \
    if constexpr (fold_tile_ok(KIND, PREC, WM_, WN_)) {                                                      \
      hipLaunchKernelGGL((fgemm_group_kernel<KIND, WM_, WN_, PREC>), grid, block, 0, st, args, tab, sources); \
      return hipGetLastError();                                                                              \
    }                                                                                                        \
    return hipErrorInvalidValue;                                                                             \
  }
  DLX_TILE(4, 4)
  DLX_TILE(3, 3)
  DLX_TILE(2, 2)
  DLX_TILE(4, 2)
  DLX_TILE(2, 4)
  DLX_TILE(2, 1)
  DLX_TILE(1, 2)
  DLX_TILE(1, 1)
  DLX_TILE(4, 1)
  DLX_TILE(1, 4)
#undef DLX_TILE
  return hipErrorInvalidValue;
}

template <int PREC>
hipError_t launch_group_prec(int kind, TileShape ts, const GemmArgs* args, const int2* tab, int n_wg,
                             const float* sources, hipStream_t st) {
  switch (kind) {
    case KIND_F1: return launch_group_kind<KIND_F1, PREC>(ts, args, tab, n_wg, sources, st);
    case KIND_F2: return launch_group_kind<KIND_F2, PREC>(ts, args, tab, n_wg, sources, st);
    case KIND_B3: return launch_group_kind<KIND_B3, PREC>(ts, args, tab, n_wg, sources, st);
    case KIND_B4: return launch_group_kind<KIND_B4, PREC>(ts, args, tab, n_wg, sources, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_gemm_group(int kind, int prec, TileShape ts, const GemmArgs* args, const int2* tab, int n_wg,
                             const float* sources, hipStream_t st) {
  if (n_wg <= 0) return hipSuccess;
  return prec == 0 ? launch_group_prec<0>(kind, ts, args, tab, n_wg, sources, st)
                   : launch_group_prec<1>(kind, ts, args, tab, n_wg, sources, st);
}

bool tile_supported(int kind, int prec, bool fold, TileShape ts) {
  for (const TileShape& t : kTileShapes)
    if (t.wm == ts.wm && t.wn == ts.wn) return !fold || fold_tile_ok(kind, prec, ts.wm, ts.wn);
  return false;
}

hipError_t launch_gemm(int kind, int prec, TileShape ts, const GemmArgs& a, int n_wg, hipStream_t st) {
  if (n_wg <= 0) return hipSuccess;
  return prec == 0 ? launch_prec<0>(kind, ts, a, n_wg, st) : launch_prec<1>(kind, ts, a, n_wg, st);
}

}  // namespace dlx
