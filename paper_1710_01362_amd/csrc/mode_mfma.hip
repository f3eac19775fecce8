// Effective-Hamiltonian contraction on the CDNA4 matrix cores.
//
// One launch handles one ModeDesc group (all terms of an H_eff apply that
// act on one bond axis with one source tensor):
//   y[s] (+)= sum_o M_{s,o} x_axis src[s + o],   M_{s,o} = sum_e coef_e g_e(s,o) E_e.
// Workgroup (blockIdx.y = output physical index s, blockIdx.x = tile of
// kModeNT "rest" columns, i.e. all indices other than the bond axis and the
// physical leg).  For every band offset o the workgroup builds the real form
//   A = [[Re M, -Im M], [Im M, Re M]]   (2D x 2D, zero-padded to DP)
// and B = [Re src; Im src] (2D x kModeNT) in LDS, and accumulates
// Y = A B on 16x16 MFMA tiles: wavefront w owns output columns 16w..16w+15
// and every row block.  Precisions:
//   FP64  : v_mfma_f64_16x16x4 (A, B and accumulation in FP64)
// Operand layouts (all three): lane l supplies A[l % 16][k-group l / 16] and
// B[k-group l / 16][l % 16]; the accumulator layouts differ (see epilogue).
//   FP32  : v_mfma_f32_16x16x4 (A, B rounded to FP32, FP32 accumulation)
//   BF16X3: v_mfma_f32_16x16x32_bf16 three times per step, x = hi + lo with
//           hi = bf16(x), lo = bf16(x - hi): hi*hi + hi*lo + lo*hi, FP32
//           accumulation.
// The epilogue stages Y through LDS, pairs real and imaginary rows and
// writes (or adds to) the FP64 output, adding the on-site term in FP64 for
// the first group of an apply.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "ttns_internal.h"

namespace ttns {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

int mode_max_bond(int prec) { return prec == TTNS_FP64 ? 48 : 64; }

namespace {

constexpr int NT = kModeNT;  // columns per workgroup (4 wavefronts x 16)

__device__ __forceinline__ unsigned short bf16_bits(float x) {
  // round to nearest even
  unsigned int u = __float_as_uint(x);
  const unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

// g_e(s, o): weight of term e for output index s reading input index s + o
__device__ __forceinline__ cd term_weight(const ModeDesc& m, int e, int s, int o, int d) {
  if (!m.op[e]) return o == 0 ? make_double2(m.coef[e], 0.0) : cz();
  if (o < m.lo[e] || o > m.hi[e] || s + o < 0 || s + o >= d) return cz();
  const cd g = m.op[e][s * d + s + o];
  return make_double2(m.coef[e] * g.x, m.coef[e] * g.y);
}

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
struct Tile;

// FP64 / FP32: A row-major [DP][DP + 1], B column-major [NT][DP + 1]
template <>
struct Tile<TTNS_FP64> {
  using T = double;
  static constexpr int DPMAX = 96, KS = 4, KPAD = 16;
};
template <>
struct Tile<TTNS_FP32> {
  using T = float;
  static constexpr int DPMAX = 128, KS = 4, KPAD = 16;
};
template <>
struct Tile<TTNS_BF16X3> {
  using T = unsigned short;  // bf16 bits, hi and lo planes
  static constexpr int DPMAX = 128, KS = 32, KPAD = 32;
};

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_mode(Op op, DevTables Tb) {
  using C = Tile<PREC>;
  using T = typename C::T;
  constexpr bool kSplit = PREC == TTNS_BF16X3;
  constexpr int LDA = C::DPMAX + (kSplit ? 8 : 1);  // row stride (elements) of A and B
  constexpr int PLANES = kSplit ? 2 : 1;
  __shared__ T As[PLANES][C::DPMAX * LDA];
  __shared__ T Bs[PLANES][NT * LDA];
  __shared__ int roff[NT];

  const ModeDesc& m = Tb.modes[op.desc];
  const Shape& sh = m.sh;
  const int ax = m.axis, pa = sh.phys_axis;
  const int D = sh.dims[ax], d = sh.dims[pa];
  const int sa = sh.stride[ax], sp = sh.stride[pa];
  const int D2 = 2 * D;
  const int DP = (D2 + C::KPAD - 1) / C::KPAD * C::KPAD;
  const int s = blockIdx.y;
  const int r0 = blockIdx.x * NT;
  const int ncol = min(NT, m.n_rest - r0);
  const cd* src = op.p0 ? op.p0 : m.src;
  cd* y = op.p1 ? op.p1 : m.y;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;

  for (int c = t; c < NT; c += kBlock) roff[c] = c < ncol ? rest_offset(sh, ax, r0 + c) : 0;

  using Acc = typename std::conditional<PREC == TTNS_FP64, d4v, f4v>::type;
  Acc acc[C::DPMAX / 16];
#pragma unroll
  for (int i = 0; i < C::DPMAX / 16; ++i) acc[i] = Acc{0, 0, 0, 0};

  for (int o = m.band_lo; o <= m.band_hi; ++o) {
    const int si = s + o;
    if (si < 0 || si >= d) continue;
    bool any = false;
    for (int e = 0; e < m.n_e; ++e) {
      const cd g = term_weight(m, e, s, o, d);
      any = any || g.x != 0.0 || g.y != 0.0;
    }
    if (!any) continue;
    __syncthreads();  // previous offset's operands are consumed
    // A = real form of M_{s,o}, zero padded to DP x DP
    for (int i = t; i < DP * DP; i += kBlock) {
      const int row = i / DP, col = i % DP;
      double v = 0.0;
      if (row < D2 && col < D2) {
        const int a = row % D, b = col % D;
        cd mm = cz();
        for (int e = 0; e < m.n_e; ++e) mm = cfma(term_weight(m, e, s, o, d), m.E[e][a * D + b], mm);
        const bool rr = row < D, cr = col < D;
        v = (rr == cr) ? mm.x : (rr ? -mm.y : mm.y);
      }
      if constexpr (kSplit) {
        const unsigned short hi = bf16_bits((float)v);
        As[0][row * LDA + col] = hi;
        As[1][row * LDA + col] = bf16_bits((float)(v - (double)bf16_float(hi)));
      } else {
        As[0][row * LDA + col] = (T)v;
      }
    }
    // B (column-major: Bs[col][k]) = [Re src; Im src] at physical index si
    const bool bfast = sa == 1;
    for (int i = t; i < DP * NT; i += kBlock) {
      int k, c;
      if (bfast) {
        k = i % DP;
        c = i / DP;
      } else {
        c = i % NT;
        k = i / NT;
      }
      double v = 0.0;
      if (k < D2 && c < ncol) {
        const cd xv = src[si * sp + (k % D) * sa + roff[c]];
        v = k < D ? xv.x : xv.y;
      }
      if constexpr (kSplit) {
        const unsigned short hi = bf16_bits((float)v);
        Bs[0][c * LDA + k] = hi;
        Bs[1][c * LDA + k] = bf16_bits((float)(v - (double)bf16_float(hi)));
      } else {
        Bs[0][c * LDA + k] = (T)v;
      }
    }
    __syncthreads();
    const int col = w * 16 + (lane & 15);
    const int kq = lane >> 4;
    for (int kk = 0; kk < DP; kk += C::KS) {
      if constexpr (kSplit) {
        const int k0 = kk + 8 * kq;
        bf8v bh, bl;
        for (int q = 0; q < 8; ++q) {
          bh[q] = __builtin_bit_cast(__bf16, Bs[0][col * LDA + k0 + q]);
          bl[q] = __builtin_bit_cast(__bf16, Bs[1][col * LDA + k0 + q]);
        }
#pragma unroll
        for (int bi = 0; bi < C::DPMAX / 16; ++bi) {
          if (bi * 16 >= DP) break;
          const int row = bi * 16 + (lane & 15);
          bf8v ah, al;
          for (int q = 0; q < 8; ++q) {
            ah[q] = __builtin_bit_cast(__bf16, As[0][row * LDA + k0 + q]);
            al[q] = __builtin_bit_cast(__bf16, As[1][row * LDA + k0 + q]);
          }
          acc[bi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[bi], 0, 0, 0);
          acc[bi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[bi], 0, 0, 0);
          acc[bi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[bi], 0, 0, 0);
        }
      } else {
        const T bv = Bs[0][col * LDA + kk + kq];
#pragma unroll
        for (int bi = 0; bi < C::DPMAX / 16; ++bi) {
          if (bi * 16 >= DP) break;
          const T av = As[0][(bi * 16 + (lane & 15)) * LDA + kk + kq];
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
  double* Ys = reinterpret_cast<double*>(&As[0][0]);  // DP x NT doubles fit in A
  {
    const int col = w * 16 + (lane & 15);
#pragma unroll
    for (int bi = 0; bi < C::DPMAX / 16; ++bi) {
      if (bi * 16 >= DP) break;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // accumulator layout: FP64 16x16x4 holds row 4q + lane/16, the FP32
        // accumulating forms hold row 4 (lane/16) + q (column lane % 16)
        const int row = PREC == TTNS_FP64 ? 4 * q + (lane >> 4) : 4 * (lane >> 4) + q;
        Ys[(bi * 16 + row) * NT + col] = (double)acc[bi][q];
      }
    }
  }
  __syncthreads();
  for (int i = t; i < D * NT; i += kBlock) {
    const int a = i / NT, c = i % NT;
    if (c >= ncol) continue;
    const int off = s * sp + a * sa + roff[c];
    cd v = make_double2(Ys[a * NT + c], Ys[(D + a) * NT + c]);
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

}  // namespace

hipError_t launch_mode(const Op& op, const DevTables& t, hipStream_t s, int prec, int n_rest, int d) {
  const dim3 grid((n_rest + NT - 1) / NT, d), block(kBlock);
  switch (prec) {
    case TTNS_FP64:
      hipLaunchKernelGGL(k_mode<TTNS_FP64>, grid, block, 0, s, op, t);
      break;
    case TTNS_FP32:
      hipLaunchKernelGGL(k_mode<TTNS_FP32>, grid, block, 0, s, op, t);
      break;
    case TTNS_BF16X3:
      hipLaunchKernelGGL(k_mode<TTNS_BF16X3>, grid, block, 0, s, op, t);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ttns
