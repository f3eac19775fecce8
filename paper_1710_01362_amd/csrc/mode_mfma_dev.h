// Device code of the matrix-core H_eff group (see mode_mfma.hip): one block
// of a group (output physical index s, a tile of rest columns) as a device
// function, shared by the group kernel and the one-workgroup executor.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "ttns_internal.h"

namespace ttns {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

namespace mfma {


__device__ __forceinline__ unsigned short bf16_bits(float x) {
  // round to nearest even
  unsigned int u = __float_as_uint(x);
  const unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

// rest column r -> tensor offset (all axes but the bond axis and the phys leg)
__device__ __forceinline__ int rest_offset(const Shape& sh, int ax, int r) {
  int off = 0;
  for (int a = sh.rank - 1; a >= 0; --a) {
    if (a == ax || a == sh.phys_axis) continue;
    off += (r % sh.dims[a]) * sh.stride[a];
    r /= sh.dims[a];
  }
  return off;
}

template <int PREC>
struct Prec;
template <>
struct Prec<TTNS_FP64> {
  using T = double;
  static constexpr int KS = 4, KPAD = 16, SMALL = 48, BIG = 96;
};
template <>
struct Prec<TTNS_FP32> {
  using T = float;
  static constexpr int KS = 4, KPAD = 16, SMALL = 64, BIG = 128;
};
template <>
struct Prec<TTNS_BF16X3> {
  using T = unsigned short;  // bf16 bits, hi and lo planes
  static constexpr int KS = 32, KPAD = 32, SMALL = 64, BIG = 128;
};

// store v (FP64) into plane 0 (and the bf16 remainder into plane 1)
template <int PREC>
__device__ __forceinline__ void put(typename Prec<PREC>::T* p0, typename Prec<PREC>::T* p1, int idx, double v) {
  if constexpr (PREC == TTNS_BF16X3) {
    const unsigned short hi = bf16_bits((float)v);
    p0[idx] = hi;
    p1[idx] = bf16_bits((float)(v - (double)bf16_float(hi)));
  } else {
    (void)p1;
    p0[idx] = (typename Prec<PREC>::T)v;
  }
}

template <int PREC, int DPMAX, int TN>
struct ModeSmem {
  using T = typename Prec<PREC>::T;
  static constexpr bool kSplit = PREC == TTNS_BF16X3;
  static constexpr int LDA = DPMAX + (kSplit ? 8 : 1);  // row stride of A and column stride of B
  static constexpr int PLANES = kSplit ? 2 : 1;
  static constexpr size_t kA = (size_t)PLANES * DPMAX * LDA * sizeof(T);
  static constexpr size_t kB = (size_t)PLANES * TN * LDA * sizeof(T);
  static constexpr size_t kY = (size_t)DPMAX * TN * sizeof(double);
  static constexpr size_t kBytes = (kA + kB > kY ? kA + kB : kY);
};

// TN: rest columns per workgroup.  TN = 64: wavefront w owns columns
// 16w..16w+15 and every row block; TN = 16: all wavefronts share the 16
// columns and wavefront w owns row blocks w, w+4, ... (four times more
// workgroups for nodes with few rest columns).
// One block of a group: output physical index s, rest columns
// [tile * TN, tile * TN + TN).  smem: S::kBytes of LDS, roff: TN ints.
template <int PREC, int DPMAX, int TN>
__device__ void mode_block(const Op& op, const DevTables& Tb, int s, int tile, unsigned char* smem, int* roff) {
  using P = Prec<PREC>;
  using S = ModeSmem<PREC, DPMAX, TN>;
  using T = typename P::T;
  constexpr bool kSplit = S::kSplit;
  constexpr int LDA = S::LDA;
  // A planes, then B planes; the epilogue reuses the space for Y (doubles)
  T* A0 = reinterpret_cast<T*>(smem);
  T* A1 = A0 + DPMAX * LDA;
  T* B0 = reinterpret_cast<T*>(smem + S::kA);
  T* B1 = B0 + TN * LDA;

  const ModeDesc& m = Tb.modes[op.desc];
  const Shape& sh = m.sh;
  const int ax = m.axis, pa = sh.phys_axis;
  const int D = sh.dims[ax], d = sh.dims[pa];
  const int sa = sh.stride[ax], sp = sh.stride[pa];
  const int D2 = 2 * D;
  const int DP = (D2 + P::KPAD - 1) / P::KPAD * P::KPAD;
  const int r0 = tile * TN;
  const int ncol = min(TN, m.n_rest - r0);
  const cd* src = op.p0 ? op.p0 : m.src;
  cd* y = op.p1 ? op.p1 : m.y;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const bool bfast = sa == 1;  // bond index fastest in memory

  for (int c = t; c < TN; c += kBlock) roff[c] = c < ncol ? rest_offset(sh, ax, r0 + c) : 0;
  // zero padding: A rows and columns >= 2D, B rows >= 2D (never rewritten)
  for (int i = t; i < DP * DP; i += kBlock) {
    const int row = i / DP, col = i % DP;
    if (row >= D2 || col >= D2) put<PREC>(A0, A1, row * LDA + col, 0.0);
  }
  for (int i = t; i < TN * (DP - D2); i += kBlock) {
    const int c = i / (DP - D2), k = D2 + i % (DP - D2);
    put<PREC>(B0, B1, c * LDA + k, 0.0);
  }

  using Acc = typename std::conditional<PREC == TTNS_FP64, d4v, f4v>::type;
  Acc acc[DPMAX / 16];
#pragma unroll
  for (int i = 0; i < DPMAX / 16; ++i) acc[i] = Acc{0, 0, 0, 0};

  constexpr int kU = ((DPMAX / 2) * TN + kBlock - 1) / kBlock;  // B elements (complex) per thread, D <= DPMAX / 2
  constexpr int kUA = (DPMAX / 2) * (DPMAX / 2) / kBlock + 1;
  const int nz = D * TN;  // complex B elements
  for (int e = 0; e < m.n_e; ++e) {
    const cd* op_e = m.op[e];
    const double coef = m.coef[e];
    const int olo = op_e ? max(m.lo[e], -s) : 0;
    const int ohi = op_e ? min(m.hi[e], d - 1 - s) : 0;
    bool any = false;
    for (int o = olo; o <= ohi; ++o) {
      const cd g = op_e ? op_e[s * d + s + o] : make_double2(1.0, 0.0);
      any = any || g.x != 0.0 || g.y != 0.0;
    }
    if (!any) continue;  // uniform: every thread read the same weights
    __syncthreads();  // the previous term's operands are consumed
    // A_e: real form of E_e, loads batched per thread
    const cd* E = m.E[e];
    {
      cd v[kUA];
#pragma unroll
      for (int u = 0; u < kUA; ++u) {
        const int i = t + u * kBlock;
        v[u] = i < D * D ? E[i] : cz();
      }
#pragma unroll
      for (int u = 0; u < kUA; ++u) {
        const int i = t + u * kBlock;
        if (i < D * D) {
          const int a = i / D, b = i % D;
          put<PREC>(A0, A1, a * LDA + b, v[u].x);
          put<PREC>(A0, A1, a * LDA + D + b, -v[u].y);
          put<PREC>(A0, A1, (D + a) * LDA + b, v[u].y);
          put<PREC>(A0, A1, (D + a) * LDA + D + b, v[u].x);
        }
      }
    }
    // B_e = Z_{e,s}: band-weighted source slices, accumulated in registers
    {
      cd z[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) z[u] = cz();
      for (int o = olo; o <= ohi; ++o) {
        const cd g = op_e ? op_e[s * d + s + o] : make_double2(1.0, 0.0);
        if (g.x == 0.0 && g.y == 0.0) continue;
        const cd wgt = make_double2(coef * g.x, coef * g.y);
        const cd* base = src + (size_t)(s + o) * sp;
        cd v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int i = t + u * kBlock;
          int b, c;
          if (bfast) {
            b = i % D;
            c = i / D;
          } else {
            c = i % TN;
            b = i / TN;
          }
          v[u] = (i < nz && c < ncol) ? base[b * sa + roff[c]] : cz();
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) z[u] = cfma(wgt, v[u], z[u]);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int i = t + u * kBlock;
        if (i < nz) {
          int b, c;
          if (bfast) {
            b = i % D;
            c = i / D;
          } else {
            c = i % TN;
            b = i / TN;
          }
          put<PREC>(B0, B1, c * LDA + b, z[u].x);
          put<PREC>(B0, B1, c * LDA + D + b, z[u].y);
        }
      }
    }
    __syncthreads();
    const int col = (TN == 64 ? w * 16 : 0) + (lane & 15);
    const int kq = lane >> 4;
    for (int kk = 0; kk < DP; kk += P::KS) {
      if constexpr (kSplit) {
        const int k0 = kk + 8 * kq;
        bf8v bh, bl;
        for (int q = 0; q < 8; ++q) {
          bh[q] = __builtin_bit_cast(__bf16, B0[col * LDA + k0 + q]);
          bl[q] = __builtin_bit_cast(__bf16, B1[col * LDA + k0 + q]);
        }
#pragma unroll
        for (int bi = 0; bi < DPMAX / 16; ++bi) {
          if (bi * 16 >= DP) break;
          if (TN == 16 && (bi & 3) != w) continue;
          const int row = bi * 16 + (lane & 15);
          bf8v ah, al;
          for (int q = 0; q < 8; ++q) {
            ah[q] = __builtin_bit_cast(__bf16, A0[row * LDA + k0 + q]);
            al[q] = __builtin_bit_cast(__bf16, A1[row * LDA + k0 + q]);
          }
          acc[bi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[bi], 0, 0, 0);
          acc[bi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[bi], 0, 0, 0);
          acc[bi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[bi], 0, 0, 0);
        }
      } else {
        const T bv = B0[col * LDA + kk + kq];
#pragma unroll
        for (int bi = 0; bi < DPMAX / 16; ++bi) {
          if (bi * 16 >= DP) break;
          if (TN == 16 && (bi & 3) != w) continue;
          const T av = A0[(bi * 16 + (lane & 15)) * LDA + kk + kq];
          if constexpr (PREC == TTNS_FP64)
            acc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[bi], 0, 0, 0);
          else
            acc[bi] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[bi], 0, 0, 0);
        }
      }
    }
  }
  __syncthreads();
  // epilogue: accumulators -> LDS (row-major Y[row][col] in double), then
  // pair real and imaginary rows
  double* Ys = reinterpret_cast<double*>(smem);
  {
    const int col = (TN == 64 ? w * 16 : 0) + (lane & 15);
#pragma unroll
    for (int bi = 0; bi < DPMAX / 16; ++bi) {
      if (bi * 16 >= DP) break;
      if (TN == 16 && (bi & 3) != w) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // accumulator layout: FP64 16x16x4 holds row 4q + lane/16, the FP32
        // accumulating forms hold row 4 (lane/16) + q (column lane % 16)
        const int row = PREC == TTNS_FP64 ? 4 * q + (lane >> 4) : 4 * (lane >> 4) + q;
        Ys[(bi * 16 + row) * TN + col] = (double)acc[bi][q];
      }
    }
  }
  __syncthreads();
  for (int i = t; i < D * TN; i += kBlock) {
    const int a = i / TN, c = i % TN;
    if (c >= ncol) continue;
    const int off = s * sp + a * sa + roff[c];
    cd v = make_double2(Ys[a * TN + c], Ys[(D + a) * TN + c]);
    if (m.accumulate) {
      v = cadd(v, y[off]);
    } else if (m.site) {
      const cd* x = op.p0 ? op.p0 : m.x;
      const int lo = max(m.site_lo, -s), hi = min(m.site_hi, d - 1 - s);
      cd part = cz();
      for (int q = lo; q <= hi; ++q) part = cfma(m.site[s * d + s + q], x[off + q * sp], part);
      v = make_double2(v.x + m.site_coef * part.x, v.y + m.site_coef * part.y);
    }
    y[off] = v;
  }
}

// Every block of a group in turn, in the calling workgroup (the
// one-workgroup executor); lds holds at least the largest tile's bytes plus
// TN ints.
template <int PREC, int DPMAX, int TN>
__device__ void mode_all_blocks(const Op& op, const DevTables& Tb, int n_rest, int d, unsigned char* lds) {
  using S = ModeSmem<PREC, DPMAX, TN>;
  int* roff = reinterpret_cast<int*>(lds + (S::kBytes + 15) / 16 * 16);
  const int tiles = (n_rest + TN - 1) / TN;
  for (int s = 0; s < d; ++s)
    for (int tile = 0; tile < tiles; ++tile) {
      mode_block<PREC, DPMAX, TN>(op, Tb, s, tile, lds, roff);
      __syncthreads();  // the next block rewrites the operands
    }
}

template <int PREC>
__device__ void mode_group_prec(const Op& op, const DevTables& Tb, int n_rest, int d, unsigned char* lds) {
  const int tile = op.i1 & 3;
  const bool small = tile == 1 || (tile == 0 && op.j <= Prec<PREC>::SMALL);
  const bool narrow = op.i1 ? (op.i1 & 4) != 0 : false;
  if (small) {
    if (narrow) mode_all_blocks<PREC, Prec<PREC>::SMALL, 16>(op, Tb, n_rest, d, lds);
    else mode_all_blocks<PREC, Prec<PREC>::SMALL, 64>(op, Tb, n_rest, d, lds);
  } else {
    if (narrow) mode_all_blocks<PREC, Prec<PREC>::BIG, 16>(op, Tb, n_rest, d, lds);
    else mode_all_blocks<PREC, Prec<PREC>::BIG, 64>(op, Tb, n_rest, d, lds);
  }
}

}  // namespace mfma
}  // namespace ttns
