// Effective-Hamiltonian contraction on the CDNA4 matrix cores.
//
// One launch handles one ModeDesc group (all terms of an H_eff apply that
// act on one bond axis with one source tensor):
//   y[s] (+)= sum_e E_e x_axis Z_{e,s},   Z_{e,s} = sum_o coef_e g_e(s,o) src[s + o],
// with g_e(s,o) = op_e[s][s + o] (the identity when the term has no local
// operator).  Workgroup (blockIdx.y = output physical index s, blockIdx.x =
// tile of 64 or 16 "rest" columns, i.e. all indices other than the bond
// axis and the physical leg).  For every term e the workgroup stages the real form
//   A_e = [[Re E_e, -Im E_e], [Im E_e, Re E_e]]   (2D x 2D, zero-padded to DP)
// and B_e = [Re Z_{e,s}; Im Z_{e,s}] (2D x columns) in LDS and accumulates
// Y += A_e B_e on 16x16 MFMA tiles (which wavefront owns which output
// tiles depends on the column tile, see k_mode).  A_e does not depend on s and B_e needs
// only the band of g_e, so every global load is a plain independent load of
// an environment matrix or a source slice, issued in batches.
// Operand layouts (all precisions): lane l supplies A[l % 16][k-group l / 16]
// and B[k-group l / 16][l % 16]; the accumulator layouts differ (epilogue).
//   FP64  : v_mfma_f64_16x16x4 (A, B and accumulation in FP64)
//   FP32  : v_mfma_f32_16x16x4 (A, B rounded to FP32, FP32 accumulation)
//   BF16X3: v_mfma_f32_16x16x32_bf16 three times per step, x = hi + lo with
//           hi = bf16(x), lo = bf16(x - hi): hi*hi + hi*lo + lo*hi, FP32
//           accumulation.
// Two tile sizes per precision: DP up to 48 (FP64) / 64 (others), whose LDS
// footprint lets several workgroups share a compute unit, and the full one.
// The epilogue stages Y through LDS, pairs real and imaginary rows and
// writes (or adds to) the FP64 output, adding the on-site term in FP64 for
// the first group of an apply.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "mode_mfma_dev.h"
#include "ttns_internal.h"

namespace ttns {

using namespace mfma;

int mode_max_bond(int prec) { return prec == TTNS_FP64 ? 48 : 64; }
int mode_small_dp(int prec) { return prec == TTNS_FP64 ? 48 : 64; }
// 16-column tiles when 64-column ones would give fewer workgroups than CUs
bool mode_default_narrow(int n_rest, int d) { return (long)((n_rest + 63) / 64) * d < 256; }
int mode_padded(int prec, int D) {
  const int pad = prec == TTNS_BF16X3 ? 32 : 16;
  return (2 * D + pad - 1) / pad * pad;
}

namespace {

template <int PREC, int DPMAX, int TN>
__global__ __launch_bounds__(kBlock) void k_mode(Op op, DevTables Tb) {
  __shared__ __align__(16) unsigned char smem[ModeSmem<PREC, DPMAX, TN>::kBytes];
  __shared__ int roff[TN];
  mode_block<PREC, DPMAX, TN>(op, Tb, blockIdx.y, blockIdx.x, smem, roff);
}

template <int PREC, int TN>
hipError_t launch_tn(const Op& op, const DevTables& t, hipStream_t s, int n_rest, int d, bool small) {
  const dim3 grid((n_rest + TN - 1) / TN, d);
  if (small)
    hipLaunchKernelGGL((k_mode<PREC, Prec<PREC>::SMALL, TN>), grid, dim3(kBlock), 0, s, op, t);
  else
    hipLaunchKernelGGL((k_mode<PREC, Prec<PREC>::BIG, TN>), grid, dim3(kBlock), 0, s, op, t);
  return hipGetLastError();
}

// op.j: padded real operand size DP of this group; op.i1: the tile chosen by
// the autotuner (bit 0: small operand tile, bit 1: large, bit 2: 16 columns
// per workgroup instead of 64) or 0 (default: the small tile when it fits,
// 16 columns when 64-column tiles would leave the GPU under-filled)
template <int PREC>
hipError_t launch_prec(const Op& op, const DevTables& t, hipStream_t s, int n_rest, int d) {
  const int tile = op.i1 & 3;
  const bool small = tile == 1 || (tile == 0 && op.j <= Prec<PREC>::SMALL);
  const bool narrow = op.i1 ? (op.i1 & 4) != 0 : mode_default_narrow(n_rest, d);
  return narrow ? launch_tn<PREC, 16>(op, t, s, n_rest, d, small) : launch_tn<PREC, 64>(op, t, s, n_rest, d, small);
}

}  // namespace

hipError_t launch_mode(const Op& op, const DevTables& t, hipStream_t s, int prec, int n_rest, int d) {
  switch (prec) {
    case TTNS_FP64:
      return launch_prec<TTNS_FP64>(op, t, s, n_rest, d);
    case TTNS_FP32:
      return launch_prec<TTNS_FP32>(op, t, s, n_rest, d);
    case TTNS_BF16X3:
      return launch_prec<TTNS_BF16X3>(op, t, s, n_rest, d);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace ttns
