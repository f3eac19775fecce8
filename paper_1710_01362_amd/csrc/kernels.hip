// Device code of the TTNS one-site TDVP step for gfx950 (CDNA4), FP64 path.
//
// Every operation of the sweep is a device function over "virtual
// workgroups" (vb = 0 .. nvb-1) of kBlock threads:
//   * the wide executor launches one kernel per operation with nvb real
//     workgroups; operations that reduce across workgroups write per-vb
//     partial sums and the last workgroup to finish (atomic ticket) folds
//     them in vb order, so results are bitwise reproducible;
//   * the persistent executor runs a whole tree's operation list inside one
//     workgroup, looping vb and calling the same fold afterwards.
//
// Complex numbers are double2 (re, im).  No floating-point atomics anywhere.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "mode_mfma_dev.h"
#include "ttns_internal.h"

namespace ttns {

// ------------------------------------------------------------ shared memory
struct Smem {
  cd red[kBlock / 64];
  cd wred[kBlock / 64][kRedStride];  // per-wavefront partial sums
  cd vec[kRedStride];                // broadcast scalars (dot products, coefficients)
  union {
    struct {
      cd M[kMaxKrylov * kMaxKrylov];  // Krylov exponential work
      cd P[kMaxKrylov * kMaxKrylov];
    } kx;
    cd lanes[kBlock];                 // wide-QR fold helpers
  };
  cd fold[64];
  int ival[4];
  double dval[4];
};

// Sum over the workgroup in a fixed order (wave butterfly, then waves 0..3).
__device__ cd block_sum(cd v, Smem& sm) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sm.red[wid] = v;
  __syncthreads();
  cd r = sm.red[0];
#pragma unroll
  for (int w = 1; w < kBlock / 64; ++w) r = cadd(r, sm.red[w]);
  return r;
}

// Two sums over the workgroup at once (same order as block_sum): returns
// the sum of a, the sum of b in *bs.
__device__ cd block_sum2(cd a, cd b, Smem& sm, cd* bs) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a.x += __shfl_xor(a.x, off);
    a.y += __shfl_xor(a.y, off);
    b.x += __shfl_xor(b.x, off);
    b.y += __shfl_xor(b.y, off);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sm.red[wid] = a;
    sm.wred[wid][0] = b;
  }
  __syncthreads();
  cd ra = sm.red[0], rb = sm.wred[0][0];
#pragma unroll
  for (int w = 1; w < kBlock / 64; ++w) {
    ra = cadd(ra, sm.red[w]);
    rb = cadd(rb, sm.wred[w][0]);
  }
  *bs = rb;
  return ra;
}

__device__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Atomic ticket: true in the workgroup that finishes last (wide executor).
// Each workgroup releases its writes before taking a ticket; the winner
// acquires before it reads the other workgroups' partial results.
__device__ bool last_block(unsigned* counter, int nvb, Smem& sm) {
  // the workgroup barrier completes every wave's stores to this CU's L2
  // path; one agent-scope release by thread 0 then publishes them all
  // (cumulative over the barrier), instead of one L2 writeback per wave
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    sm.ival[0] = (prev == (unsigned)(nvb - 1));
    if (sm.ival[0]) atomicExch(counter, 0u);
  }
  __syncthreads();
  const bool last = sm.ival[0] != 0;
  if (last) __threadfence();
  return last;
}

// ------------------------------------------------------------ H_eff apply
__device__ __forceinline__ int coord(const Shape& sh, int idx, int a) {
  return (idx / sh.stride[a]) % sh.dims[a];
}

// One output element of y = site o x + sum_e coef_e op_e o E_e (src_e),
// computed by the 2^lg consecutive lanes that share idx: lane `sub` takes
// every 2^lg-th term of each contraction loop, and butterflies add the
// shares (every lane of the group returns the sum).  Spreading a small node
// over more lanes shortens each lane's chain of dependent loads.
__device__ cd apply_point(const ApplyDesc& d, const cd* __restrict__ x, int idx, int sub, int lg) {
  const int G = 1 << lg;
  const Shape& sh = d.sh;
  const int pa = sh.phys_axis;
  const int dp = sh.dims[pa], sp = sh.stride[pa];
  const int s = coord(sh, idx, pa);
  cd acc = cz();
  if (d.site) {
    const int lo = max(d.site_lo, -s), hi = min(d.site_hi, dp - 1 - s);
    cd part = cz();
    for (int o = lo + sub; o <= hi; o += G) part = cfma(d.site[s * dp + s + o], x[idx + o * sp], part);
    acc = cscale(part, d.site_coef);
  }
  for (int k = 0; k < d.n_entries; ++k) {
    const Entry& e = d.e[k];
    const cd* __restrict__ src = e.src < 0 ? x : d.tmp[e.src];
    const int D = sh.dims[e.axis], st = sh.stride[e.axis];
    const int a = coord(sh, idx, e.axis);
    const int base = idx - a * st;
    const cd* __restrict__ Erow = e.E + a * D;
    cd part = cz();
    if (!e.op) {
      for (int b = sub; b < D; b += G) part = cfma(Erow[b], src[base + b * st], part);
    } else {
      const int lo = max(e.op_lo, -s), hi = min(e.op_hi, dp - 1 - s);
      for (int o = lo; o <= hi; ++o) {
        const cd oc = e.op[s * dp + s + o];
        const cd* __restrict__ sb = src + base + o * sp;
        cd inner = cz();
        for (int b = sub; b < D; b += G) inner = cfma(Erow[b], sb[b * st], inner);
        part = cfma(oc, inner, part);
      }
    }
    acc.x = fma(e.coef, part.x, acc.x);
    acc.y = fma(e.coef, part.y, acc.y);
  }
  for (int off = G >> 1; off > 0; off >>= 1) {
    acc.x += __shfl_xor(acc.x, off);
    acc.y += __shfl_xor(acc.y, off);
  }
  return acc;
}

// Element and lane of this thread in an apply over 2^lg lanes per element.
__device__ __forceinline__ int apply_idx(int vb, int lg) { return vb * (kBlock >> lg) + (int)(threadIdx.x >> lg); }
__device__ __forceinline__ int apply_sub(int lg) { return (int)(threadIdx.x & ((1u << lg) - 1u)); }

// OP_APPLY: desc.y = H x with x = op.p0 when given (Lanczos pre-stages read
// the current Krylov vector), else desc.x; op.i1 = lg (2^lg lanes per
// element).
__device__ void body_apply(const Op& op, const DevTables& T, int vb) {
  const ApplyDesc& d = T.descs[op.desc];
  const cd* x = op.p0 ? op.p0 : d.x;
  const int lg = op.i1;
  const int idx = apply_idx(vb, lg), sub = apply_sub(lg);
  if (idx < d.sh.size) {
    const cd y = apply_point(d, x, idx, sub, lg);
    if (sub == 0) d.y[idx] = y;
  }
}

// ------------------------------------------------------------ Lanczos pieces
// Partial sums of conj(V_i) . w (i = 0..j) and |w|^2 of this vb: every
// thread forms its j+2 products, each wavefront reduces them by butterflies,
// and the four wavefront sums are added in order.
__device__ void lz_partials(const TreeDev& tr, int j, int n, int vb, int idx, cd w, cd* part, Smem& sm) {
  constexpr int kChunk = 6;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int cnt = j + 2;
  for (int c0 = 0; c0 < cnt; c0 += kChunk) {  // uniform trip count
    cd val[kChunk];
#pragma unroll
    for (int q = 0; q < kChunk; ++q) {
      const int i = c0 + q;
      val[q] = cz();
      if (idx < n) {
        if (i <= j) val[q] = cjfma(tr.V[(size_t)i * tr.ldv + idx], w, val[q]);
        else if (i == j + 1) val[q].x = cabs2(w);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        val[q].x += __shfl_xor(val[q].x, off);
        val[q].y += __shfl_xor(val[q].y, off);
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < kChunk; ++q)
        if (c0 + q < kRedStride) sm.wred[wid][c0 + q] = val[q];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    cd s = sm.wred[0][threadIdx.x];
#pragma unroll
    for (int w2 = 1; w2 < kBlock / 64; ++w2) s = cadd(s, sm.wred[w2][threadIdx.x]);
    part[vb * kRedStride + threadIdx.x] = s;
  }
  __syncthreads();
}

// Fold the partial sums of the previous Lanczos op (nvb workgroups x cnt
// values, stride kRedStride) into sm.vec[0..cnt-1].  Every workgroup of the
// consuming op folds for itself, in the same fixed order (kFoldSeg
// segments of workgroups summed in parallel, then the segments in order),
// so no workgroup of the producer waits for the others.
constexpr int kFoldSeg = kBlock / kRedStride;
__device__ void lz_fold(const cd* __restrict__ part, int nvb, int cnt, Smem& sm) {
  const int t = threadIdx.x;
  const int seg = t / kRedStride, i = t - seg * kRedStride;
  if (seg < kFoldSeg && i < cnt) {
    cd s = cz();
#pragma unroll 6
    for (int b = seg; b < nvb; b += kFoldSeg) s = cadd(s, part[b * kRedStride + i]);
    sm.lanes[seg * kRedStride + i] = s;
  }
  __syncthreads();
  if (t < cnt) {
    cd s = sm.lanes[t];
    for (int g = 1; g < kFoldSeg; ++g) s = cadd(s, sm.lanes[g * kRedStride + t]);
    sm.vec[t] = s;
  }
  __syncthreads();
}

// OP_NORM: |x| of the vector about to be evolved (op.p0, op.n elements).
__device__ void body_norm(const Op& op, const DevTables& T, int vb, Smem& sm) {
  const TreeDev& tr = T.trees[op.tree];
  const int idx = vb * kBlock + threadIdx.x;
  cd q = make_double2(idx < op.n ? cabs2(op.p0[idx]) : 0.0, 0.0);
  q = block_sum(q, sm);
  if (threadIdx.x == 0) tr.partials[vb * kRedStride] = q;
}
__device__ void fin_norm(const Op& op, const DevTables& T, int nvb, Smem& sm) {
  const TreeDev& tr = T.trees[op.tree];
  cd part = cz();
  for (int b = threadIdx.x; b < nvb; b += kBlock) part = cadd(part, tr.partials[b * kRedStride]);
  const double s = block_sum(part, sm).x;
  if (threadIdx.x == 0) {
    const double nx = sqrt(s);
    tr.scal->nx = nx;
    tr.scal->inv_nx = nx > 0.0 ? 1.0 / nx : 0.0;
    tr.scal->done = nx > 0.0 ? 0 : 1;
    tr.scal->k_eff = 0;
  }
}

// OP_SCALE: V_0 = x / |x|
__device__ void body_scale(const Op& op, const DevTables& T, int vb) {
  const TreeDev& tr = T.trees[op.tree];
  const int idx = vb * kBlock + threadIdx.x;
  if (idx < op.n) tr.V[idx] = cscale(op.p0[idx], tr.scal->inv_nx);
}

// OP_APPLY_LZ: W = H V_j and its partial dots.  Returns false when the
// Lanczos process already stopped (uniform over all workgroups).
__device__ bool body_apply_lz(const Op& op, const DevTables& T, int vb, Smem& sm) {
  const TreeDev& tr = T.trees[op.tree];
  if (tr.scal->done) return false;
  const ApplyDesc& d = T.descs[op.desc];
  const int n = d.sh.size;
  const int lg = op.i1;  // 0 when the matrix-core groups produced W
  const int idx = apply_idx(vb, lg), sub = apply_sub(lg);
  cd w = cz();
  if (idx < n) {
    if (op.i0) {  // W was produced by the matrix-core groups of this apply
      w = tr.W[idx];
    } else {
      w = apply_point(d, tr.V + (size_t)op.j * tr.ldv, idx, sub, lg);
      if (sub == 0) tr.W[idx] = w;
    }
  }
  // one lane per element enters the dots
  lz_partials(tr, op.j, n, vb, sub == 0 ? idx : n, sub == 0 ? w : cz(), op.p1, sm);
  return true;
}

// OP_ORTH1: first classical Gram-Schmidt pass, partial dots of the result.
// Prologue (once per workgroup, before its vbs): h1 = V^H W from the
// partials of OP_APPLY_LZ (op.p2, op.i0 workgroups) into sm.vec; `keep`:
// this workgroup also stores h1 for alpha_j.
__device__ void orth1_prologue(const Op& op, const DevTables& T, Smem& sm, bool keep) {
  const TreeDev& tr = T.trees[op.tree];
  lz_fold(op.p2, op.i0, op.j + 2, sm);
  if (keep && (int)threadIdx.x <= op.j) tr.scal->h1[threadIdx.x] = sm.vec[threadIdx.x];
}
__device__ void body_orth1(const Op& op, const DevTables& T, int vb, Smem& sm) {
  const TreeDev& tr = T.trees[op.tree];
  const int n = op.n, j = op.j;
  const int idx = vb * kBlock + threadIdx.x;
  cd w = cz();
  if (idx < n) {
    w = tr.W[idx];
    for (int i = 0; i <= j; ++i) {
      const cd h = sm.vec[i];
      const cd v = tr.V[(size_t)i * tr.ldv + idx];
      w = csub(w, make_double2(h.x * v.x - h.y * v.y, h.x * v.y + h.y * v.x));
    }
    tr.W[idx] = w;
  }
  lz_partials(tr, j, n, vb, idx, w, op.p1, sm);
}

// OP_ORTH2 prologue: h2 = V^H W and |W|^2 after the first pass, from the
// partials of OP_ORTH1 (op.p2, op.i0 workgroups), into sm.vec.
__device__ void orth2_prologue(const Op& op, Smem& sm) { lz_fold(op.p2, op.i0, op.j + 2, sm); }

// beta_j from the second pass (same value in every workgroup): |W|^2 after
// the second subtraction by the norm identity.
__device__ double lz_beta(const Smem& sm, int j) {
  double b2 = sm.vec[j + 1].x;
  for (int i = 0; i <= j; ++i) b2 -= cabs2(sm.vec[i]);
  return sqrt(fmax(b2, 0.0));
}
__device__ bool lz_stop(const TreeDev& tr, const Op& op, double beta) {
  const int j = op.j;
  return (j == tr.kmax - 1) || (j == op.n - 1) || (beta <= tr.btol * tr.scal->nx);
}

// OP_ORTH2: second pass, beta_j, V_{j+1} (unless the process stops here).
__device__ void body_orth2(const Op& op, const DevTables& T, int vb, const Smem& sm) {
  const TreeDev& tr = T.trees[op.tree];
  const int n = op.n, j = op.j;
  const double beta = lz_beta(sm, j);
  if (lz_stop(tr, op, beta)) return;
  const double ib = 1.0 / beta;
  const int idx = vb * kBlock + threadIdx.x;
  if (idx < n) {
    cd w = tr.W[idx];
    for (int i = 0; i <= j; ++i) {
      const cd h = sm.vec[i];
      const cd v = tr.V[(size_t)i * tr.ldv + idx];
      w = csub(w, make_double2(h.x * v.x - h.y * v.y, h.x * v.y + h.y * v.x));
    }
    tr.V[(size_t)(j + 1) * tr.ldv + idx] = cscale(w, ib);
  }
}
// alpha_j, beta_j and the stop decision (one workgroup).
__device__ void fin_orth2(const Op& op, const DevTables& T, const Smem& sm) {
  const TreeDev& tr = T.trees[op.tree];
  LzScal* sc = tr.scal;
  if (threadIdx.x == 0) {
    const int j = op.j;
    const double beta = lz_beta(sm, j);
    sc->alpha[j] = sc->h1[j].x + sm.vec[j].x;
    if (lz_stop(tr, op, beta)) {
      sc->k_eff = j + 1;
      sc->done = 1;
      if (j < tr.kmax - 1 && j < op.n - 1) atomicAdd(&tr.stats[1], 1);
    } else {
      sc->beta[j] = beta;
    }
  }
}

// exp(i zim T) e_1 for the k x k real symmetric tridiagonal T = (alpha,
// beta): scaling and squaring with an 18-term Taylor series of the scaled
// matrix (|i zim T / 2^q| <= 1/2).  Result in sm.vec[0..k-1]; all threads.
__device__ void krylov_exp(const double* alpha, const double* beta, int k, double zim, Smem& sm) {
  const int t = threadIdx.x;
  if (t < 64) {
    double nb = 0.0;
    if (t < k) {
      nb = fabs(alpha[t]);
      if (t > 0) nb += fabs(beta[t - 1]);
      if (t + 1 < k) nb += fabs(beta[t]);
    }
    nb = wave_max(nb) * fabs(zim);
    if (t == 0) {
      int q = 0;
      double sc = 1.0;
      while (nb * sc > 0.5 && q < 60) {
        sc *= 0.5;
        ++q;
      }
      sm.ival[1] = q;
      sm.dval[0] = sc;
    }
  }
  __syncthreads();
  const int q = sm.ival[1];
  const double zs = zim * sm.dval[0];
  const int r = t / kMaxKrylov, c = t % kMaxKrylov;
  const bool mine = (t < kMaxKrylov * kMaxKrylov) && r < k && c < k;
  // P = I, M = I
  if (t < kMaxKrylov * kMaxKrylov) {
    cd one = make_double2((r == c) ? 1.0 : 0.0, 0.0);
    sm.kx.P[t] = one;
    sm.kx.M[t] = one;
  }
  __syncthreads();
  for (int term = 1; term <= 18; ++term) {
    // P <- P (i zs T) / term
    cd v = cz();
    if (mine) {
      cd acc = cz();
      if (c > 0) acc = cscale(sm.kx.P[r * kMaxKrylov + c - 1], beta[c - 1]);
      acc = cadd(acc, cscale(sm.kx.P[r * kMaxKrylov + c], alpha[c]));
      if (c + 1 < k) acc = cadd(acc, cscale(sm.kx.P[r * kMaxKrylov + c + 1], beta[c]));
      const double f = zs / (double)term;
      v = make_double2(-acc.y * f, acc.x * f);  // i * f * acc
    }
    __syncthreads();
    if (mine) {
      sm.kx.P[r * kMaxKrylov + c] = v;
      sm.kx.M[r * kMaxKrylov + c] = cadd(sm.kx.M[r * kMaxKrylov + c], v);
    }
    __syncthreads();
  }
  for (int sq = 0; sq < q; ++sq) {
    cd v = cz();
    if (mine)
      for (int m = 0; m < k; ++m) v = cfma(sm.kx.M[r * kMaxKrylov + m], sm.kx.M[m * kMaxKrylov + c], v);
    __syncthreads();
    if (mine) sm.kx.M[r * kMaxKrylov + c] = v;
    __syncthreads();
  }
  if (t < k) sm.vec[t] = sm.kx.M[t * kMaxKrylov];
  __syncthreads();
}

// OP_COMBINE: out = |x| sum_i c_i V_i with c = exp(sign i h T) e_1.
__device__ void body_combine(const Op& op, const DevTables& T, int vb, Smem& sm) {
  const TreeDev& tr = T.trees[op.tree];
  const LzScal* sc = tr.scal;
  const int k = sc->k_eff;
  const double h = *T.half_step;
  if (k > 0) krylov_exp(sc->alpha, sc->beta, k, op.sign * h, sm);
  const int idx = vb * kBlock + threadIdx.x;
  if (idx < op.n) {
    cd acc = cz();
    for (int i = 0; i < k; ++i) acc = cfma(sm.vec[i], tr.V[(size_t)i * tr.ldv + idx], acc);
    op.p1[idx] = cscale(acc, sc->nx);
  }
}

// ------------------------------------------------------------ guarded QR
// Row r of the matricisation towards `ax` (other axes row-major in axis
// order) -> tensor offset with column 0.
__device__ int qr_row_offset(const Shape& sh, int ax, int r) {
  int off = 0;
  for (int a = sh.rank - 1; a >= 0; --a) {
    if (a == ax) continue;
    const int c = r % sh.dims[a];
    r /= sh.dims[a];
    off += c * sh.stride[a];
  }
  return off;
}

// Completion candidate n (physical index fastest, then the other bond axes
// in axis order) -> row index of the matricisation towards `ax`.
__device__ int qr_candidate_row(const Shape& sh, int ax, int n) {
  int row = 0;
  // row-major stride of axis a among the rows = product of later non-ax dims
  auto rstride = [&](int a) {
    int s = 1;
    for (int b = a + 1; b < sh.rank; ++b)
      if (b != ax) s *= sh.dims[b];
    return s;
  };
  const int pa = sh.phys_axis;
  if (pa != ax) {
    row += (n % sh.dims[pa]) * rstride(pa);
    n /= sh.dims[pa];
  }
  for (int a = 0; a < sh.rank; ++a) {
    if (a == ax || a == pa) continue;
    row += (n % sh.dims[a]) * rstride(a);
    n /= sh.dims[a];
  }
  return row;
}

// h[j] = sum_r conj(Q_j[r]) v[r] for j < k (waves take columns, lanes rows).
__device__ void qr_project(const cd* Q, const cd* v, int rows, int k, cd* h) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j = wid; j < k; j += kBlock / 64) {
    const cd* q = Q + (size_t)j * rows;
    cd a0 = cz(), a1 = cz();  // two chains keep several loads in flight
    int r = lane;
#pragma unroll 2
    for (; r + 64 < rows; r += 128) {
      a0 = cjfma(q[r], v[r], a0);
      a1 = cjfma(q[r + 64], v[r + 64], a1);
    }
    if (r < rows) a0 = cjfma(q[r], v[r], a0);
    cd acc = cadd(a0, a1);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off);
      acc.y += __shfl_xor(acc.y, off);
    }
    if (lane == 0) h[j] = acc;
  }
  __syncthreads();
}

// v[r] -= sum_j Q_j[r] h[j]; returns this thread's share of |v|^2.
// sync = false: the caller's next step begins with a workgroup barrier.
__device__ double qr_subtract(const cd* Q, cd* v, int rows, int k, const cd* h, bool sync = true) {
  double n2 = 0.0;
  for (int r = threadIdx.x; r < rows; r += kBlock) {
    cd a0 = v[r], a1 = cz();
    int j = 0;
#pragma unroll 2
    for (; j + 1 < k; j += 2) {
      const cd q0 = Q[(size_t)j * rows + r], q1 = Q[(size_t)(j + 1) * rows + r];
      const cd h0 = h[j], h1 = h[j + 1];
      a0 = csub(a0, make_double2(q0.x * h0.x - q0.y * h0.y, q0.x * h0.y + q0.y * h0.x));
      a1 = csub(a1, make_double2(q1.x * h1.x - q1.y * h1.y, q1.x * h1.y + q1.y * h1.x));
    }
    if (j < k) {
      const cd q0 = Q[(size_t)j * rows + r];
      const cd h0 = h[j];
      a0 = csub(a0, make_double2(q0.x * h0.x - q0.y * h0.y, q0.x * h0.y + q0.y * h0.x));
    }
    const cd acc = cadd(a0, a1);
    v[r] = acc;
    n2 += cabs2(acc);
  }
  if (sync) __syncthreads();
  return n2;
}

constexpr int kQrWRows = 640;  // rows whose span weights the QR keeps in LDS (what the LDS budget leaves)

// LDS budget of the QR (complex entries): Q columns plus two row vectors.
constexpr int kQrLds = kQrLdsEntries;  // 137.5 KiB: a 400 x 20 matrix plus two vectors

// OP_QR (one workgroup): node tensor op.p1 (shape of desc op.desc) = Q R
// towards axis op.axis; Q overwrites the tensor, R -> tree R buffer.
// Column-by-column classical Gram-Schmidt applied twice; a column whose
// residual is <= rank_tol |A|_F is replaced by the first unit vector (in
// completion order) farther than half the average from the span so far,
// orthogonalised twice.  Q and the work vectors live in LDS (`lds`, kQrLds
// entries) when they fit, else in the tree's global scratch.
template <bool kLds>
__device__ void body_qr_t(const Op& op, const DevTables& T, Smem& sm, cd* lds, double* wrow,
                          unsigned short* ctab) {
  const TreeDev& tr = T.trees[op.tree];
  const Shape& sh = T.descs[op.desc].sh;
  const int ax = op.axis;
  const int cols = sh.dims[ax];
  const int rows = sh.size / cols;
  const int cst = sh.stride[ax];
  cd* Q = kLds ? lds : tr.qrQ;
  // with LDS, A is gathered into Q's own buffer: column k of A is read (into
  // registers, one column ahead) before column k of Q overwrites it
  cd* A = kLds ? lds : tr.qrA;
  cd* v = kLds ? lds + (size_t)rows * cols : tr.qrv;
  cd* u = kLds ? v + rows : tr.qrv + tr.max_rows;
  cd* R = tr.R;
  cd* X = op.p1;
  __shared__ cd hb1[64], hb2[64];
  // gather A (column-major), |A|_F^2 and the squared norm of every column
  __shared__ double colnrm[64];
  // wrow[r] = sum_{j<k} |Q_j[r]|^2, kept up to date as columns are finished
  // (when rows <= kQrWRows), so the completion search reads one number per
  // candidate instead of k
  const bool track = wrow != nullptr && rows <= kQrWRows;
  for (int c = threadIdx.x; c < cols; c += kBlock) colnrm[c] = 0.0;
  __syncthreads();
  for (int r = threadIdx.x; r < rows; r += kBlock) {
    const int off = qr_row_offset(sh, ax, r);
    for (int c = 0; c < cols; ++c) {
      const cd a = X[off + c * cst];
      A[(size_t)c * rows + r] = a;
    }
  }
  __syncthreads();
  {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c = wid; c < cols; c += kBlock / 64) {
      double s = 0.0;
      for (int r = lane; r < rows; r += 64) s += cabs2(A[(size_t)c * rows + r]);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
      if (lane == 0) colnrm[c] = s;
    }
  }
  for (int i = threadIdx.x; i < cols * cols; i += kBlock) R[i] = cz();
  if (track)
    for (int r = threadIdx.x; r < rows; r += kBlock) {
      wrow[r] = 0.0;
      ctab[r] = (unsigned short)qr_candidate_row(sh, ax, r);  // completion order -> row
    }
  __syncthreads();
  double nrm = 0.0;
  for (int c = 0; c < cols; ++c) nrm += colnrm[c];
  const double tol = tr.rtol * sqrt(nrm);
  // each thread owns rows tid, tid + kBlock, ...; the next column of A is
  // loaded into registers while the current one is processed
  constexpr int kPre = 4;
  cd nxt[kPre];
#pragma unroll
  for (int i = 0; i < kPre; ++i) {
    const int r = threadIdx.x + i * kBlock;
    nxt[i] = r < rows ? A[r] : cz();
  }
  // a finished column k is written to Q (q_k = v / rn) in the next
  // iteration's load phase, by the thread owning each row, before that
  // thread loads the next column into v: one barrier for both
  int pend_k = -1;
  double pend_ir = 0.0;
  auto write_pending = [&]() {
    if (pend_k < 0) return;
    cd* qp = Q + (size_t)pend_k * rows;
    for (int r = threadIdx.x; r < rows; r += kBlock) {
      const cd q = cscale(v[r], pend_ir);
      qp[r] = q;
      if (track) wrow[r] += cabs2(q);
    }
    pend_k = -1;
  };
  for (int k = 0; k < cols; ++k) {
    write_pending();
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
      const int r = threadIdx.x + i * kBlock;
      if (r < rows) v[r] = nxt[i];
    }
    for (int r = threadIdx.x + kPre * kBlock; r < rows; r += kBlock) v[r] = A[(size_t)k * rows + r];
    if (k + 1 < cols) {
#pragma unroll
      for (int i = 0; i < kPre; ++i) {
        const int r = threadIdx.x + i * kBlock;
        if (r < rows) nxt[i] = A[(size_t)(k + 1) * rows + r];
      }
    }
    __syncthreads();
    // a column no longer than tol is deficient whatever its projections:
    // one pass gives its R entries and residual; otherwise two passes
    const bool tiny = sqrt(colnrm[k]) <= tol;
    double rn;
    if (colnrm[k] == 0.0) {
      // an exactly zero column: every projection and the residual are
      // exactly zero, as the passes below would compute them
      for (int j = threadIdx.x; j < k; j += kBlock) hb1[j] = hb2[j] = cz();
      rn = 0.0;
      __syncthreads();
    } else if (tiny) {
      qr_project(Q, v, rows, k, hb1);
      rn = sqrt(block_sum(make_double2(qr_subtract(Q, v, rows, k, hb1, false), 0.0), sm).x);
      for (int j = threadIdx.x; j < k; j += kBlock) hb2[j] = cz();
      __syncthreads();
    } else {
      qr_project(Q, v, rows, k, hb1);
      qr_subtract(Q, v, rows, k, hb1);
      qr_project(Q, v, rows, k, hb2);
      rn = sqrt(block_sum(make_double2(qr_subtract(Q, v, rows, k, hb2, false), 0.0), sm).x);
    }
    for (int j = threadIdx.x; j < k; j += kBlock) R[j * cols + k] = cadd(hb1[j], hb2[j]);
    cd* qk = Q + (size_t)k * rows;
    if (rn > tol) {
      if (threadIdx.x == 0) R[k * cols + k] = make_double2(rn, 0.0);
      pend_k = k;
      pend_ir = 1.0 / rn;
      continue;
    }
    // completion: first candidate with distance^2 > (rows - k) / (2 rows),
    // kBlock candidates per round
    const double thr = 0.5 * (double)(rows - k) / (double)rows;
    {
      __shared__ int wfirst[kBlock / 64];
      const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
      int chosen = -1;
      for (int base = 0; base < rows && chosen < 0; base += kBlock) {
        const int n = base + (int)threadIdx.x;
        bool ok = false;
        if (n < rows) {
          const int row = track ? ctab[n] : qr_candidate_row(sh, ax, n);
          double w;
          if (track) {
            w = wrow[row];
          } else {
            double s = 0.0, s1 = 0.0;
            int j = 0;
#pragma unroll 2
            for (; j + 1 < k; j += 2) {
              s += cabs2(Q[(size_t)j * rows + row]);
              s1 += cabs2(Q[(size_t)(j + 1) * rows + row]);
            }
            if (j < k) s += cabs2(Q[(size_t)j * rows + row]);
            w = s + s1;
          }
          ok = (1.0 - w) > thr;
        }
        const unsigned long long m = __ballot(ok);
        if (lane == 0) wfirst[wid] = m ? base + wid * 64 + __ffsll((long long)m) - 1 : -1;
        __syncthreads();
        for (int w2 = 0; w2 < kBlock / 64 && chosen < 0; ++w2) chosen = wfirst[w2];
        __syncthreads();
      }
      if (threadIdx.x == 0)
        sm.ival[2] = chosen < 0 ? -1 : track ? ctab[chosen] : qr_candidate_row(sh, ax, chosen);
    }
    __syncthreads();
    const int row = sm.ival[2];
    if (row < 0) {
      if (threadIdx.x == 0) atomicOr(&tr.stats[3], 1);  // cannot happen for rows >= cols
      return;
    }
    // u = e_row - Q (Q^H e_row), then a second pass
    bool nz = false;
    for (int j = threadIdx.x; j < k; j += kBlock) {
      const cd q = Q[(size_t)j * rows + row];
      hb1[j] = make_double2(q.x, -q.y);
      nz = nz || q.x != 0.0 || q.y != 0.0;
    }
    if (!__syncthreads_or(nz)) {
      // e_row is exactly orthogonal to the span (every coefficient is zero,
      // as for the unit columns of product-like states): the general path
      // below would give q_k = e_row and R_kk = <e_row, v> = v[row] exactly
      for (int r = threadIdx.x; r < rows; r += kBlock) {
        qk[r] = make_double2(r == row ? 1.0 : 0.0, 0.0);
        if (track && r == row) wrow[r] += 1.0;
      }
      if (threadIdx.x == 0) {
        R[k * cols + k] = v[row];
        atomicAdd(&tr.stats[0], 1);
      }
      __syncthreads();
      continue;
    }
    // u = e_row - Q h (the projection coefficients of a unit vector are
    // read, not computed, so one pass leaves u orthogonal to the span to
    // ~k eps / |u|); |u|^2 and u^H v in one reduction: q_k = u / |u|,
    // R_kk = u^H v / |u|
    double uu = 0.0;
    cd uv = cz();
    for (int r = threadIdx.x; r < rows; r += kBlock) {
      cd a0 = make_double2(r == row ? 1.0 : 0.0, 0.0), a1 = cz();
      int j = 0;
#pragma unroll 2
      for (; j + 1 < k; j += 2) {
        const cd q0 = Q[(size_t)j * rows + r], q1 = Q[(size_t)(j + 1) * rows + r];
        const cd h0 = hb1[j], h1 = hb1[j + 1];
        a0 = csub(a0, make_double2(q0.x * h0.x - q0.y * h0.y, q0.x * h0.y + q0.y * h0.x));
        a1 = csub(a1, make_double2(q1.x * h1.x - q1.y * h1.y, q1.x * h1.y + q1.y * h1.x));
      }
      if (j < k) {
        const cd q0 = Q[(size_t)j * rows + r];
        const cd h0 = hb1[j];
        a0 = csub(a0, make_double2(q0.x * h0.x - q0.y * h0.y, q0.x * h0.y + q0.y * h0.x));
      }
      a0 = cadd(a0, a1);
      u[r] = a0;
      uu += cabs2(a0);
      uv = cjfma(a0, v[r], uv);
    }
    const cd red = block_sum2(make_double2(uu, 0.0), uv, sm, &uv);
    const double iu = 1.0 / sqrt(red.x);
    for (int r = threadIdx.x; r < rows; r += kBlock) {
      const cd q = cscale(u[r], iu);
      qk[r] = q;
      if (track) wrow[r] += cabs2(q);
    }
    if (threadIdx.x == 0) {
      R[k * cols + k] = cscale(uv, iu);
      atomicAdd(&tr.stats[0], 1);
    }
    __syncthreads();
  }
  write_pending();
  __syncthreads();
  // scatter Q back into the node tensor
  for (int r = threadIdx.x; r < rows; r += kBlock) {
    const int off = qr_row_offset(sh, ax, r);
    for (int c = 0; c < cols; ++c) X[off + c * cst] = Q[(size_t)c * rows + r];
  }
}

// kTrack: keep the span weights and the completion-order table in LDS (the
// wide executor's QR kernel); the one-workgroup executors' kernels hold
// other LDS buffers and do without.
template <bool kTrack>
__device__ void body_qr(const Op& op, const DevTables& T, Smem& sm, cd* lds) {
  const Shape& sh = T.descs[op.desc].sh;
  const int cols = sh.dims[op.axis];
  const int rows = sh.size / cols;
  double* wrow = nullptr;
  unsigned short* ctab = nullptr;
  if constexpr (kTrack) {
    __shared__ double w[kQrWRows];
    __shared__ unsigned short ct[kQrWRows];
    wrow = w;
    ctab = ct;
  }
  if ((size_t)rows * (cols + 2) <= (size_t)kQrLds) body_qr_t<true>(op, T, sm, lds, wrow, ctab);
  else body_qr_t<false>(op, T, sm, nullptr, wrow, ctab);
}

// ------------------------------------------------------------ fast QR
// The guarded QR of body_qr_t (classical Gram-Schmidt applied twice, column
// by column, the same completion rule) organised for latency in one
// workgroup of kQrThreads threads with Q in LDS.  Thread t owns rows
// t, t + kQrThreads, ... (at most kQrRpt) and keeps their residual of the
// current column in registers.  A projection Q^H v gives every coefficient
// j a group of L lanes of one wavefront (L = 64, 32, 16 or 8, the widest
// that leaves a group for every coefficient): the lanes sum interleaved
// rows with four independent chains and a butterfly adds the lanes.  The
// second pass also carries |v|^2, so that |v2|^2 = |v1|^2 - |h2|^2 (the
// Pythagorean identity of the projection) needs no reduction of its own.
// A completion vector u = e_row - Q Q^H e_row needs no reduction either:
// |u|^2 = 1 - sum_j |Q_j[row]|^2 is the row's span weight, and
// u^H v = v[row] up to rounding (v is orthogonal to the span).  Column k of
// A is read from the node tensor one column ahead.

// Workgroup barrier for data exchanged through LDS only: waits for this
// wave's LDS operations but not for its global loads still in flight (so a
// prefetch of the next column is not drained at every barrier, as the full
// __syncthreads() fence would do).  The kernels using it exchange nothing
// through global memory inside the workgroup.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// h[j] = sum_r conj(Q_j[r]) x[r] for j < k and, with `norm`, h[k] = |x|^2;
// x = vb (LDS) or, with Q == nullptr, column j of the node tensor X (the
// column norms at the start: every slot is a norm).  Ends with h visible.
template <int L>
__device__ void qf_slots(const cd* Q, const cd* vb, const cd* X, const int* roff, int cst, int rows, int k,
                         int ns, cd* h) {
  const int t = threadIdx.x;
  const int j = t / L, g = t % L;
  cd s0 = cz(), s1 = cz(), s2 = cz(), s3 = cz();
  if (j < ns) {
    if (!Q) {  // squared norm of tensor column j
      int r = g;
      for (; r + 3 * L < rows; r += 4 * L) {
        s0.x += cabs2(X[roff[r] + j * cst]);
        s1.x += cabs2(X[roff[r + L] + j * cst]);
        s2.x += cabs2(X[roff[r + 2 * L] + j * cst]);
        s3.x += cabs2(X[roff[r + 3 * L] + j * cst]);
      }
      for (; r < rows; r += L) s0.x += cabs2(X[roff[r] + j * cst]);
    } else if (j < k) {
      const cd* q = Q + (size_t)j * rows;
      int r = g;
      for (; r + 3 * L < rows; r += 4 * L) {
        s0 = cjfma(q[r], vb[r], s0);
        s1 = cjfma(q[r + L], vb[r + L], s1);
        s2 = cjfma(q[r + 2 * L], vb[r + 2 * L], s2);
        s3 = cjfma(q[r + 3 * L], vb[r + 3 * L], s3);
      }
      for (; r < rows; r += L) s0 = cjfma(q[r], vb[r], s0);
    } else {  // j == k: |vb|^2
      int r = g;
      for (; r + 3 * L < rows; r += 4 * L) {
        s0.x += cabs2(vb[r]);
        s1.x += cabs2(vb[r + L]);
        s2.x += cabs2(vb[r + 2 * L]);
        s3.x += cabs2(vb[r + 3 * L]);
      }
      for (; r < rows; r += L) s0.x += cabs2(vb[r]);
    }
  }
  cd s = cadd(cadd(s0, s1), cadd(s2, s3));
#pragma unroll
  for (int off = L >> 1; off > 0; off >>= 1) {
    s.x += __shfl_xor(s.x, off);
    s.y += __shfl_xor(s.y, off);
  }
  if (g == 0 && j < ns) h[j] = s;
  lds_barrier();
}
__device__ void qf_project(const cd* Q, const cd* vb, const cd* X, const int* roff, int cst, int rows, int k,
                           int ns, cd* h) {
  if (ns <= kQrThreads / 64) qf_slots<64>(Q, vb, X, roff, cst, rows, k, ns, h);
  else if (ns <= kQrThreads / 32) qf_slots<32>(Q, vb, X, roff, cst, rows, k, ns, h);
  else if (ns <= kQrThreads / 16) qf_slots<16>(Q, vb, X, roff, cst, rows, k, ns, h);
  else qf_slots<8>(Q, vb, X, roff, cst, rows, k, ns, h);
}

// w - sum_{j<k} Q_j[r] c[j] with four independent chains
__device__ __forceinline__ cd qf_sub(const cd* Q, int rows, int r, int k, const cd* c, cd w) {
  cd w1 = cz(), w2 = cz(), w3 = cz();
  int j = 0;
  for (; j + 3 < k; j += 4) {
    const cd q0 = Q[(size_t)j * rows + r], q1 = Q[(size_t)(j + 1) * rows + r];
    const cd q2 = Q[(size_t)(j + 2) * rows + r], q3 = Q[(size_t)(j + 3) * rows + r];
    w = csub(w, make_double2(q0.x * c[j].x - q0.y * c[j].y, q0.x * c[j].y + q0.y * c[j].x));
    w1 = csub(w1, make_double2(q1.x * c[j + 1].x - q1.y * c[j + 1].y, q1.x * c[j + 1].y + q1.y * c[j + 1].x));
    w2 = csub(w2, make_double2(q2.x * c[j + 2].x - q2.y * c[j + 2].y, q2.x * c[j + 2].y + q2.y * c[j + 2].x));
    w3 = csub(w3, make_double2(q3.x * c[j + 3].x - q3.y * c[j + 3].y, q3.x * c[j + 3].y + q3.y * c[j + 3].x));
  }
  for (; j < k; ++j) {
    const cd q0 = Q[(size_t)j * rows + r];
    w = csub(w, make_double2(q0.x * c[j].x - q0.y * c[j].y, q0.x * c[j].y + q0.y * c[j].x));
  }
  return cadd(cadd(w, w1), cadd(w2, w3));
}

__global__ __launch_bounds__(kQrThreads) void k_qr_fast(Op op, DevTables T) {
  __shared__ __align__(16) unsigned char lds[kQrFastLds];
  __shared__ int wfirst[kQrThreads / 64];
  const TreeDev& tr = T.trees[op.tree];
  const Shape& sh = T.descs[op.desc].sh;
  const int ax = op.axis;
  const int cols = sh.dims[ax], rows = sh.size / cols, cst = sh.stride[ax];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  cd* Q = reinterpret_cast<cd*>(lds);   // column-major Q[c * rows + r]
  cd* vb = Q + (size_t)rows * cols;    // residual of the current column
  cd* h1 = vb + rows;                  // first-pass coefficients [0, 66)
  cd* h2 = h1 + 66;                    // second pass [0, k) and |v1|^2 at [k]
  cd* cn = h2 + 66;                    // column norms (real parts) [0, 64)
  double* wrow = reinterpret_cast<double*>(cn + 64);  // sum_{j<k} |Q_j[r]|^2
  int* roff = reinterpret_cast<int*>(wrow + rows);
  unsigned short* ctab = reinterpret_cast<unsigned short*>(roff + rows);
  cd* R = tr.R;
  cd* X = op.p1;
  for (int r = t; r < rows; r += kQrThreads) {
    roff[r] = qr_row_offset(sh, ax, r);
    wrow[r] = 0.0;
    ctab[r] = (unsigned short)qr_candidate_row(sh, ax, r);
  }
  for (int i = t; i < cols * cols; i += kQrThreads) R[i] = cz();
  __syncthreads();  // a full barrier: the zeroed R entries land before any thread writes one
  qf_project(nullptr, nullptr, X, roff, cst, rows, 0, cols, cn);
  double nrm = 0.0;
  for (int c = 0; c < cols; ++c) nrm += cn[c].x;
  const double tol = tr.rtol * sqrt(nrm);
  cd a[kQrRpt], v[kQrRpt];
#pragma unroll
  for (int i = 0; i < kQrRpt; ++i) {
    const int r = t + i * kQrThreads;
    a[i] = r < rows ? X[roff[r]] : cz();
  }
  for (int k = 0; k < cols; ++k) {
#pragma unroll
    for (int i = 0; i < kQrRpt; ++i) v[i] = a[i];
    if (k + 1 < cols) {  // the next column's loads stay in flight
#pragma unroll
      for (int i = 0; i < kQrRpt; ++i) {
        const int r = t + i * kQrThreads;
        a[i] = r < rows ? X[roff[r] + (k + 1) * cst] : cz();
      }
    }
    const double c2 = cn[k].x;
    double rn = 0.0;
    if (c2 != 0.0 && k == 0) {
      rn = sqrt(c2);
    } else if (c2 != 0.0) {
      // first pass
#pragma unroll
      for (int i = 0; i < kQrRpt; ++i) {
        const int r = t + i * kQrThreads;
        if (r < rows) vb[r] = v[i];
      }
      lds_barrier();
      qf_project(Q, vb, nullptr, nullptr, 0, rows, k, k, h1);
#pragma unroll
      for (int i = 0; i < kQrRpt; ++i) {
        const int r = t + i * kQrThreads;
        if (r < rows) v[i] = qf_sub(Q, rows, r, k, h1, v[i]);
      }
      // a column no longer than tol is deficient whatever its projections:
      // one pass gives its R entries and residual
      if (sqrt(c2) > tol) {
        lds_barrier();  // every thread has read vb
#pragma unroll
        for (int i = 0; i < kQrRpt; ++i) {
          const int r = t + i * kQrThreads;
          if (r < rows) vb[r] = v[i];
        }
        lds_barrier();
        qf_project(Q, vb, nullptr, nullptr, 0, rows, k, k + 1, h2);
        double hh = 0.0;
        for (int j = 0; j < k; ++j) hh += cabs2(h2[j]);
        rn = sqrt(fmax(h2[k].x - hh, 0.0));
#pragma unroll
        for (int i = 0; i < kQrRpt; ++i) {
          const int r = t + i * kQrThreads;
          if (r < rows) v[i] = qf_sub(Q, rows, r, k, h2, v[i]);
        }
        if (t < k) R[t * cols + k] = cadd(h1[t], h2[t]);
      } else if (t < k) {
        R[t * cols + k] = h1[t];
      }
    }
    cd* qk = Q + (size_t)k * rows;
    if (rn > tol) {
      const double ir = 1.0 / rn;
#pragma unroll
      for (int i = 0; i < kQrRpt; ++i) {
        const int r = t + i * kQrThreads;
        if (r >= rows) continue;
        const cd q = cscale(v[i], ir);
        qk[r] = q;
        wrow[r] += cabs2(q);
      }
      if (t == 0) R[k * cols + k] = make_double2(rn, 0.0);
      continue;  // the next column's first barrier orders these writes
    }
    // completion: first candidate (completion order) whose squared distance
    // from the span exceeds (rows - k) / (2 rows)
    lds_barrier();  // wrow of every row is current; h1 / h2 are consumed
    const double thr = 0.5 * (double)(rows - k) / (double)rows;
    int chosen = -1;
    for (int base = 0; base < rows && chosen < 0; base += kQrThreads) {
      const int n = base + t;
      const bool ok = n < rows && (1.0 - wrow[ctab[n]]) > thr;
      const unsigned long long m = __ballot(ok);
      if (lane == 0) wfirst[wid] = m ? base + wid * 64 + __ffsll((long long)m) - 1 : -1;
      lds_barrier();
      for (int w2 = 0; w2 < kQrThreads / 64 && chosen < 0; ++w2) chosen = wfirst[w2];
      lds_barrier();
    }
    if (chosen < 0) {  // no candidate: a non-finite matrix (rows >= cols otherwise)
      if (t == 0) atomicOr(&tr.stats[3], 1);
      return;
    }
    const int row = ctab[chosen];
    // coefficients conj(Q_j[row]) of the unit vector e_row
    bool nz = false;
    for (int j = t; j < k; j += kQrThreads) {
      const cd q = Q[(size_t)j * rows + row];
      h1[j] = make_double2(q.x, -q.y);
      nz = nz || q.x != 0.0 || q.y != 0.0;
    }
    const double iu = 1.0 / sqrt(1.0 - wrow[row]);  // read before the row's weight changes
    if (!__syncthreads_or(nz)) {
      // e_row is exactly orthogonal to the span: q_k = e_row, R_kk = v[row]
#pragma unroll
      for (int i = 0; i < kQrRpt; ++i) {
        const int r = t + i * kQrThreads;
        if (r >= rows) continue;
        qk[r] = make_double2(r == row ? 1.0 : 0.0, 0.0);
        if (r == row) {
          wrow[r] += 1.0;
          R[k * cols + k] = v[i];
        }
      }
    } else {
      // q_k = (e_row - Q h) / |u|, R_kk = <q_k, v> = v[row] / |u|
#pragma unroll
      for (int i = 0; i < kQrRpt; ++i) {
        const int r = t + i * kQrThreads;
        if (r >= rows) continue;
        const cd u = qf_sub(Q, rows, r, k, h1, make_double2(r == row ? 1.0 : 0.0, 0.0));
        const cd q = cscale(u, iu);
        qk[r] = q;
        wrow[r] += cabs2(q);
        if (r == row) R[k * cols + k] = cscale(v[i], iu);
      }
    }
    if (t == 0) atomicAdd(&tr.stats[0], 1);
    lds_barrier();  // h1 is rewritten by the next column
  }
  lds_barrier();
  // scatter Q back into the node tensor (row owners)
  for (int r = t; r < rows; r += kQrThreads) {
    const int off = roff[r];
    for (int c = 0; c < cols; ++c) X[off + c * cst] = Q[(size_t)c * rows + r];
  }
}

// ------------------------------------------------------------ wide QR
// The same column-by-column CGS2 with completion as body_qr, for matrices
// too large for one workgroup's LDS, as a sequence of launches over row
// chunks (vb).  Phases (op.i0), column k = op.j:
//   0 gather A, |A|_F^2                      (fold: tol, zero R)
//   1 finalise Q_{k-1} (v/rn or u*iu; k > 0), v = A_k, partial Q^H A_k
//   2 v -= Q h1, partial Q^H v
//   3 v -= Q h2, partial |v|^2               (fold: rn, R column, decision)
//   4 completion only: every workgroup scans for the first admissible unit
//     vector (same answer everywhere), u = e_row - Q (Q^H e_row), partial Q^H u
//   5 completion only: u -= Q h2, partial |u|^2 and <u|v>  (fold: R_kk, iu)
//   6 finalise the last column and scatter Q into the node tensor.
__device__ void qrw_rows(const Op& op, int rows, int vb, int& r0, int& r1) {
  const int chunk = (rows + op.nvb - 1) / op.nvb;
  r0 = vb * chunk;
  r1 = min(rows, r0 + chunk);
}

// partial[j] = sum_{r in chunk} conj(Q_j[r]) x[r], j < k (waves take columns).
__device__ void qrw_project(const TreeDev& tr, const cd* Q, const cd* x, int rows, int k, int r0,
                            int r1, int vb) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j = wid; j < k; j += kBlock / 64) {
    const cd* q = Q + (size_t)j * rows;
    cd acc = cz();
    for (int r = r0 + lane; r < r1; r += 64) acc = cjfma(q[r], x[r], acc);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off);
      acc.y += __shfl_xor(acc.y, off);
    }
    if (lane == 0) tr.qrpart[vb * kQrStride + j] = acc;
  }
}

// Fold slots [0, cnt) of the wide-QR partial sums over all workgroups into
// sm.fold[0..cnt) (every thread takes (slot, workgroup) pairs, then one
// thread per slot adds the kBlock / cnt partial lanes in order).
__device__ void qrw_fold_all(const TreeDev& tr, int nvb, int cnt, Smem& sm) {
  const int t = threadIdx.x;
  const int lanes = cnt > 0 ? kBlock / cnt : 1;  // helpers per slot
  const int s = t / lanes, l = t % lanes;
  if (cnt > 0 && s < cnt) {
    cd acc = cz();
    for (int b = l; b < nvb; b += lanes) acc = cadd(acc, tr.qrpart[b * kQrStride + s]);
    sm.lanes[t] = acc;
  }
  __syncthreads();
  if (t < cnt) {
    cd acc = cz();
    for (int q = 0; q < lanes; ++q) acc = cadd(acc, sm.lanes[t * lanes + q]);
    sm.fold[t] = acc;
  }
  __syncthreads();
}

// Finalise column c of Q in this chunk from the previous column's outcome.
__device__ void qrw_finalise(const TreeDev& tr, cd* Q, int rows, int c, int r0, int r1) {
  const QrScal* s = tr.qrs;
  const cd* src = s->deficient ? tr.qrv + tr.max_rows : tr.qrv;
  const double f = s->deficient ? s->iu : 1.0 / s->rn;
  for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) Q[(size_t)c * rows + r] = cscale(src[r], f);
}

// Returns true when the phase did work that needs a fold (uniform).
__device__ bool body_qrw(const Op& op, const DevTables& T, int vb, Smem& sm) {
  const TreeDev& tr = T.trees[op.tree];
  const Shape& sh = T.descs[op.desc].sh;
  const int ax = op.axis, cols = sh.dims[ax], rows = sh.size / cols, cst = sh.stride[ax];
  const int k = op.j;
  cd* A = tr.qrA;
  cd* Q = tr.qrQ;
  cd* v = tr.qrv;
  cd* u = tr.qrv + tr.max_rows;
  int r0, r1;
  qrw_rows(op, rows, vb, r0, r1);
  QrScal* s = tr.qrs;
  switch (op.i0) {
    case 0: {
      double n2 = 0.0;
      for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) {
        const int off = qr_row_offset(sh, ax, r);
        for (int c = 0; c < cols; ++c) {
          const cd a = op.p1[off + c * cst];
          A[(size_t)c * rows + r] = a;
          n2 += cabs2(a);
        }
      }
      n2 = block_sum(make_double2(n2, 0.0), sm).x;
      if (threadIdx.x == 0) tr.qrpart[vb * kQrStride] = make_double2(n2, 0.0);
      return true;
    }
    case 1: {
      if (k > 0) qrw_finalise(tr, Q, rows, k - 1, r0, r1);
      const cd* a = A + (size_t)k * rows;
      for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) v[r] = a[r];
      __syncthreads();
      qrw_project(tr, Q, a, rows, k, r0, r1, vb);
      return true;
    }
    case 2:
    case 3: {
      const cd* h = op.i0 == 2 ? s->h1 : s->h2;
      double n2 = 0.0;
      for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) {
        cd acc = v[r];
        for (int j = 0; j < k; ++j) {
          const cd q = Q[(size_t)j * rows + r];
          const cd hj = h[j];
          acc = csub(acc, make_double2(q.x * hj.x - q.y * hj.y, q.x * hj.y + q.y * hj.x));
        }
        v[r] = acc;
        n2 += cabs2(acc);
      }
      __syncthreads();
      if (op.i0 == 2) {
        qrw_project(tr, Q, v, rows, k, r0, r1, vb);
      } else {
        n2 = block_sum(make_double2(n2, 0.0), sm).x;
        if (threadIdx.x == 0) tr.qrpart[vb * kQrStride] = make_double2(n2, 0.0);
      }
      return true;
    }
    case 4: {
      if (!s->deficient) return false;
      const double thr = 0.5 * (double)(rows - k) / (double)rows;
      if (threadIdx.x < 64) {
        int chosen = -1;
        for (int base = 0; base < rows && chosen < 0; base += 64) {
          const int n = base + (int)threadIdx.x;
          bool ok = false;
          if (n < rows) {
            const int row = qr_candidate_row(sh, ax, n);
            double t = 0.0;
            for (int j = 0; j < k; ++j) t += cabs2(Q[(size_t)j * rows + row]);
            ok = (1.0 - t) > thr;
          }
          const unsigned long long m = __ballot(ok);
          if (m) chosen = base + __ffsll((long long)m) - 1;
        }
        if (threadIdx.x == 0) sm.ival[2] = chosen < 0 ? -1 : qr_candidate_row(sh, ax, chosen);
      }
      __syncthreads();
      const int row = sm.ival[2];
      if (row < 0) {
        if (threadIdx.x == 0 && vb == 0) atomicOr(&tr.stats[3], 1);
        return true;
      }
      for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) {
        cd acc = make_double2(r == row ? 1.0 : 0.0, 0.0);
        for (int j = 0; j < k; ++j) {
          const cd q = Q[(size_t)j * rows + r];
          const cd g = Q[(size_t)j * rows + row];  // coefficient conj(Q_j[row])
          acc = csub(acc, make_double2(q.x * g.x + q.y * g.y, -q.x * g.y + q.y * g.x));
        }
        u[r] = acc;
      }
      __syncthreads();
      if (vb == 0 && threadIdx.x == 0) s->row = row;
      qrw_project(tr, Q, u, rows, k, r0, r1, vb);
      return true;
    }
    case 5: {
      if (!s->deficient) return false;
      cd nu = cz(), uv = cz();
      for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) {
        cd acc = u[r];
        for (int j = 0; j < k; ++j) {
          const cd q = Q[(size_t)j * rows + r];
          const cd hj = s->h2[j];
          acc = csub(acc, make_double2(q.x * hj.x - q.y * hj.y, q.x * hj.y + q.y * hj.x));
        }
        u[r] = acc;
        nu.x += cabs2(acc);
        uv = cjfma(acc, v[r], uv);
      }
      nu = block_sum(nu, sm);
      uv = block_sum(uv, sm);
      if (threadIdx.x == 0) {
        tr.qrpart[vb * kQrStride] = nu;
        tr.qrpart[vb * kQrStride + 1] = uv;
      }
      return true;
    }
    case 6: {
      qrw_finalise(tr, Q, rows, cols - 1, r0, r1);
      __syncthreads();
      for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) {
        const int off = qr_row_offset(sh, ax, r);
        for (int c = 0; c < cols; ++c) op.p1[off + c * cst] = Q[(size_t)c * rows + r];
      }
      return false;
    }
  }
  return false;
}

__device__ void fin_qrw(const Op& op, const DevTables& T, int nvb, Smem& sm) {
  const TreeDev& tr = T.trees[op.tree];
  const Shape& sh = T.descs[op.desc].sh;
  const int cols = sh.dims[op.axis];
  const int k = op.j;
  QrScal* s = tr.qrs;
  cd* R = tr.R;
  const int t = threadIdx.x;
  const int cnt = (op.i0 == 1 || op.i0 == 2 || op.i0 == 4) ? k : (op.i0 == 5 ? 2 : 1);
  qrw_fold_all(tr, nvb, cnt, sm);
  switch (op.i0) {
    case 0:
      for (int i = t; i < cols * cols; i += kBlock) R[i] = cz();
      if (t == 0) s->tol = tr.rtol * sqrt(sm.fold[0].x);
      break;
    case 1:
      if (t < k) s->h1[t] = sm.fold[t];
      break;
    case 2:
      if (t < k) s->h2[t] = sm.fold[t];
      break;
    case 3:
      if (t < k) R[t * cols + k] = cadd(s->h1[t], s->h2[t]);
      if (t == 0) {
        const double rn = sqrt(sm.fold[0].x);
        s->rn = rn;
        s->deficient = rn > s->tol ? 0 : 1;
        if (!s->deficient) R[k * cols + k] = make_double2(rn, 0.0);
      }
      break;
    case 4:
      if (t < k) s->h2[t] = sm.fold[t];
      break;
    case 5:
      if (t == 0) {
        const double nu = sqrt(sm.fold[0].x);
        const cd uv = sm.fold[1];
        s->iu = 1.0 / nu;
        R[k * cols + k] = cscale(uv, s->iu);
        atomicAdd(&tr.stats[0], 1);
      }
      break;
  }
}

// ------------------------------------------------------------ contraction
// OP_CONTRACT: E[a', a] = sum_r conj(Qm[r, a']) Zm[r, a] over the rows of
// the matricisations towards op.axis; Q = op.p0, Z = op.p2, shape from
// desc.  Output op.p1 (D x D, row-major) or, with op.i0 = 1, transposed
// into the current record at double offset op.i1.  Rows are split over vb.
// Rows of this vb are staged in LDS (kCtRows at a time: Q and Z rows of D
// entries each), then every thread accumulates its (a', a) pairs from LDS.
constexpr int kCtRows = 32;
__device__ void body_contract(const Op& op, const DevTables& T, int vb, Smem& sm, cd* lds) {
  const TreeDev& tr = T.trees[op.tree];
  const Shape& sh = T.descs[op.desc].sh;
  const int ax = op.axis;
  const int D = sh.dims[ax], st = sh.stride[ax];
  const int rows = sh.size / D;
  const int chunk = (rows + op.nvb - 1) / op.nvb;
  const int r0 = vb * chunk, r1 = min(rows, r0 + chunk);
  cd* part = tr.cpart + (size_t)vb * D * D;  // per-vb partial matrix
  cd* qs = lds;                    // kCtRows x D
  cd* zs = lds + kCtRows * 64;     // kCtRows x D
  constexpr int kPairs = 16;       // D <= 64: at most 4096 pairs, 16 per thread
  cd acc[kPairs];
#pragma unroll
  for (int q = 0; q < kPairs; ++q) acc[q] = cz();
  for (int base = r0; base < r1; base += kCtRows) {
    const int nb = min(kCtRows, r1 - base);
    __syncthreads();
    for (int e = threadIdx.x; e < nb * D; e += kBlock) {
      const int i = e / D, a = e % D;
      const int off = qr_row_offset(sh, ax, base + i) + a * st;
      qs[i * D + a] = op.p0[off];
      zs[i * D + a] = op.p2[off];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPairs; ++q) {
      const int p = threadIdx.x + q * kBlock;
      if (p < D * D) {
        const int a1 = p / D, a2 = p % D;
        cd s = acc[q];
        for (int i = 0; i < nb; ++i) s = cjfma(qs[i * D + a1], zs[i * D + a2], s);
        acc[q] = s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kPairs; ++q) {
    const int p = threadIdx.x + q * kBlock;
    if (p < D * D) part[p] = acc[q];
  }
}
__device__ void fin_contract(const Op& op, const DevTables& T, int nvb) {
  const TreeDev& tr = T.trees[op.tree];
  const Shape& sh = T.descs[op.desc].sh;
  const int D = sh.dims[op.axis];
  for (int p = threadIdx.x; p < D * D; p += kBlock) {
    cd s = cz();
#pragma unroll 8
    for (int b = 0; b < nvb; ++b) s = cadd(s, tr.cpart[(size_t)b * D * D + p]);
    if (op.i0 == 0) {
      op.p1[p] = s;
    } else {
      const int slot = min(*tr.rec_count, tr.rec_cap - 1);
      double* rec = tr.hist + (size_t)slot * tr.rec_size + op.i1;
      const int a1 = p / D, a2 = p % D;
      rec[2 * (a2 * D + a1)] = s.x;
      rec[2 * (a2 * D + a1) + 1] = s.y;
    }
  }
}

// ------------------------------------------------------------ bond step
// Y = H_b X for the bond matrix X (Du x Dv), one workgroup; scratch S (Du x Dv).
// The environment matrices come from `st` (LDS copies laid out as Eu, Ev^T,
// then Eu_k, Ev_k^T per pair) when staged, else from the descriptor.
__device__ __forceinline__ const cd* bond_mat(const BondDesc& b, const cd* st, int which, int k) {
  const int u2 = b.Du * b.Du, v2 = b.Dv * b.Dv;
  if (!st) return which == 0 ? (k < 0 ? b.Eu : b.Euk[k]) : (k < 0 ? b.Ev : b.Evk[k]);
  const int pair = k < 0 ? 0 : k + 1;
  return st + (size_t)pair * (u2 + v2) + (which == 0 ? 0 : u2);
}

// Products of the staged bond step, all operands row-major in LDS, 2 x 2
// output blocks per thread (each loaded entry feeds two products):
//   MODE 0: Y = A1 B1 + A2 B2,   MODE 1: Y += coef A1 B1
// with A1 (Du x K1), B1 (K1 x Dv), A2 (Du x K2), B2 (K2 x Dv), Y (Du x Dv).
// Rows / columns past the edge of an odd dimension are computed from the
// last row / column and not stored.  Ends with a barrier.
template <int MODE>
__device__ void bond_mm(int Du, int Dv, const cd* A1, const cd* B1, int K1, const cd* A2, const cd* B2, int K2,
                        cd* Y, double coef) {
  const int bu = (Du + 1) >> 1, bv = (Dv + 1) >> 1;
  for (int t = threadIdx.x; t < bu * bv; t += kBlock) {
    const int a0 = 2 * (t / bv), c0 = 2 * (t % bv);
    const int a1 = min(a0 + 1, Du - 1), c1 = min(c0 + 1, Dv - 1);
    cd y00 = cz(), y01 = cz(), y10 = cz(), y11 = cz();
#pragma unroll 4
    for (int m = 0; m < K1; ++m) {
      const cd p0 = A1[a0 * K1 + m], p1 = A1[a1 * K1 + m];
      const cd q0 = B1[m * Dv + c0], q1 = B1[m * Dv + c1];
      y00 = cfma(p0, q0, y00);
      y01 = cfma(p0, q1, y01);
      y10 = cfma(p1, q0, y10);
      y11 = cfma(p1, q1, y11);
    }
    if (MODE == 0) {
#pragma unroll 4
      for (int m = 0; m < K2; ++m) {
        const cd p0 = A2[a0 * K2 + m], p1 = A2[a1 * K2 + m];
        const cd q0 = B2[m * Dv + c0], q1 = B2[m * Dv + c1];
        y00 = cfma(p0, q0, y00);
        y01 = cfma(p0, q1, y01);
        y10 = cfma(p1, q0, y10);
        y11 = cfma(p1, q1, y11);
      }
    }
    auto put = [&](int a, int c, cd v) {
      cd* o = Y + a * Dv + c;
      if (MODE == 0) *o = v;
      else *o = make_double2(fma(coef, v.x, o->x), fma(coef, v.y, o->y));
    };
    put(a0, c0, y00);
    if (c0 + 1 < Dv) put(a0, c0 + 1, y01);
    if (a0 + 1 < Du) {
      put(a0 + 1, c0, y10);
      if (c0 + 1 < Dv) put(a0 + 1, c0 + 1, y11);
    }
  }
  __syncthreads();
}

// Every pair at once (S holds n_pairs scratch matrices): S_k = X Ev_k^T for
// all k in one pass, then Y += sum_k coef_k Eu_k S_k in one pass, adding
// the pairs in order as the one-pair-at-a-time form does.
__device__ void bond_pairs(const BondDesc& b, const cd* st, const cd* X, cd* Y, cd* S) {
  const int Du = b.Du, Dv = b.Dv, n = Du * Dv, np = b.n_pairs;
  const int bu = (Du + 1) >> 1, bv = (Dv + 1) >> 1;
  for (int t = threadIdx.x; t < bu * bv * np; t += kBlock) {
    const int k = t / (bu * bv), tb = t - k * bu * bv;
    const int a0 = 2 * (tb / bv), c0 = 2 * (tb % bv);
    const int a1 = min(a0 + 1, Du - 1), c1 = min(c0 + 1, Dv - 1);
    const cd* B = bond_mat(b, st, 1, k);
    cd y00 = cz(), y01 = cz(), y10 = cz(), y11 = cz();
#pragma unroll 4
    for (int m = 0; m < Dv; ++m) {
      const cd p0 = X[a0 * Dv + m], p1 = X[a1 * Dv + m];
      const cd q0 = B[m * Dv + c0], q1 = B[m * Dv + c1];
      y00 = cfma(p0, q0, y00);
      y01 = cfma(p0, q1, y01);
      y10 = cfma(p1, q0, y10);
      y11 = cfma(p1, q1, y11);
    }
    cd* o = S + (size_t)k * n;
    o[a0 * Dv + c0] = y00;
    if (c0 + 1 < Dv) o[a0 * Dv + c0 + 1] = y01;
    if (a0 + 1 < Du) {
      o[(a0 + 1) * Dv + c0] = y10;
      if (c0 + 1 < Dv) o[(a0 + 1) * Dv + c0 + 1] = y11;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < bu * bv; t += kBlock) {
    const int a0 = 2 * (t / bv), c0 = 2 * (t % bv);
    const int a1 = min(a0 + 1, Du - 1), c1 = min(c0 + 1, Dv - 1);
    cd y00 = Y[a0 * Dv + c0], y01 = Y[a0 * Dv + c1], y10 = Y[a1 * Dv + c0], y11 = Y[a1 * Dv + c1];
    for (int k = 0; k < np; ++k) {
      const cd* A = bond_mat(b, st, 0, k);
      const cd* Sk = S + (size_t)k * n;
      cd p00 = cz(), p01 = cz(), p10 = cz(), p11 = cz();
#pragma unroll 4
      for (int m = 0; m < Du; ++m) {
        const cd e0 = A[a0 * Du + m], e1 = A[a1 * Du + m];
        const cd q0 = Sk[m * Dv + c0], q1 = Sk[m * Dv + c1];
        p00 = cfma(e0, q0, p00);
        p01 = cfma(e0, q1, p01);
        p10 = cfma(e1, q0, p10);
        p11 = cfma(e1, q1, p11);
      }
      const double c = b.coef[k];
      y00 = make_double2(fma(c, p00.x, y00.x), fma(c, p00.y, y00.y));
      y01 = make_double2(fma(c, p01.x, y01.x), fma(c, p01.y, y01.y));
      y10 = make_double2(fma(c, p10.x, y10.x), fma(c, p10.y, y10.y));
      y11 = make_double2(fma(c, p11.x, y11.x), fma(c, p11.y, y11.y));
    }
    Y[a0 * Dv + c0] = y00;
    if (c0 + 1 < Dv) Y[a0 * Dv + c0 + 1] = y01;
    if (a0 + 1 < Du) {
      Y[(a0 + 1) * Dv + c0] = y10;
      if (c0 + 1 < Dv) Y[(a0 + 1) * Dv + c0 + 1] = y11;
    }
  }
  __syncthreads();
}

// all_pairs: S has room for n_pairs matrices (bond_pairs), else one.
__device__ void bond_apply(const BondDesc& b, const cd* st, const cd* X, cd* Y, cd* S, bool all_pairs) {
  const int Du = b.Du, Dv = b.Dv, n = Du * Dv;
  if (st && all_pairs) {
    bond_mm<0>(Du, Dv, bond_mat(b, st, 0, -1), X, Du, X, bond_mat(b, st, 1, -1), Dv, Y, 0.0);
    if (b.n_pairs > 0) bond_pairs(b, st, X, Y, S);
    return;
  }
  if (st) {
    // staged: Ev and Evk are held transposed, so X Ev^T reads rows of both
    bond_mm<0>(Du, Dv, bond_mat(b, st, 0, -1), X, Du, X, bond_mat(b, st, 1, -1), Dv, Y, 0.0);
    for (int k = 0; k < b.n_pairs; ++k) {
      bond_mm<0>(Du, Dv, X, bond_mat(b, st, 1, k), Dv, nullptr, nullptr, 0, S, 0.0);
      bond_mm<1>(Du, Dv, bond_mat(b, st, 0, k), S, Du, nullptr, nullptr, 0, Y, b.coef[k]);
    }
    return;
  }
  const cd* Eu = bond_mat(b, st, 0, -1);
  const cd* Ev = bond_mat(b, st, 1, -1);
  for (int p = threadIdx.x; p < n; p += kBlock) {
    const int a = p / Dv, c = p % Dv;
    cd acc = cz();
    for (int m = 0; m < Du; ++m) acc = cfma(Eu[a * Du + m], X[m * Dv + c], acc);
    for (int m = 0; m < Dv; ++m) acc = cfma(X[a * Dv + m], Ev[c * Dv + m], acc);
    Y[p] = acc;
  }
  __syncthreads();
  for (int k = 0; k < b.n_pairs; ++k) {
    const cd* Euk = bond_mat(b, st, 0, k);
    const cd* Evk = bond_mat(b, st, 1, k);
    for (int p = threadIdx.x; p < n; p += kBlock) {
      const int a = p / Dv, c = p % Dv;
      cd acc = cz();
      for (int m = 0; m < Dv; ++m) acc = cfma(X[a * Dv + m], Evk[c * Dv + m], acc);
      S[p] = acc;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < n; p += kBlock) {
      const int a = p / Dv, c = p % Dv;
      cd acc = cz();
      for (int m = 0; m < Du; ++m) acc = cfma(Euk[a * Du + m], S[m * Dv + c], acc);
      Y[p] = make_double2(fma(b.coef[k], acc.x, Y[p].x), fma(b.coef[k], acc.y, Y[p].y));
    }
    __syncthreads();
  }
}

// hh[i] = V_i^H W for i < cnt (cnt <= 16; V with leading dimension ld, W of
// n entries): 16 lanes per dot each sum a strided share, butterflies add the
// shares; all dots at once, one barrier.
__device__ void bond_dots(const cd* V, int ld, const cd* W, int n, int cnt, cd* hh) {
  constexpr int L = kBlock / kMaxKrylov;
  const int i = threadIdx.x / L, seg = threadIdx.x % L;
  cd d = cz();
  if (i < cnt)
    for (int p = seg; p < n; p += L) d = cjfma(V[(size_t)i * ld + p], W[p], d);
#pragma unroll
  for (int off = L >> 1; off > 0; off >>= 1) {
    d.x += __shfl_xor(d.x, off);
    d.y += __shfl_xor(d.y, off);
  }
  if (i < cnt && seg == 0) hh[i] = d;
  __syncthreads();
}

// LDS entries of a staged bond step: Krylov basis, W, `scratch` matrices
// and the environment matrices.
__device__ size_t bond_lds_need(const BondDesc& b, int kmax, int scratch) {
  const size_t n = (size_t)b.Du * b.Dv;
  return (kmax + 2 + scratch) * n + (size_t)(1 + b.n_pairs) * (b.Du * b.Du + b.Dv * b.Dv);
}

// OP_BOND (one workgroup): R <- exp(sign i h H_b) R by the same Lanczos
// process as the nodes (CGS2, breakdown, Krylov dimension kmax).  The
// Krylov basis, work vectors and environment matrices are staged in LDS
// (`lds`, kQrLds entries) when they fit, else used from global memory.
template <bool kLds>
__device__ void body_bond_t(const Op& op, const DevTables& T, Smem& sm, cd* lds) {
  const TreeDev& tr = T.trees[op.tree];
  const BondDesc& b = T.bonds[op.desc];
  const int n = b.Du * b.Dv;
  const int kmax = min(tr.kmax, n);
  const int ld = kLds ? n : op.i0;  // leading dimension of the Krylov basis
  cd* V = kLds ? lds : tr.bondV;
  cd* W = kLds ? lds + (size_t)(kmax + 1) * n : tr.bondW;
  cd* S = kLds ? W + n : tr.bondW + op.i0;
  // room in LDS for one scratch matrix per pair
  const bool all_pairs = kLds && bond_lds_need(b, kmax, max(b.n_pairs, 1)) <= (size_t)kQrLds;
  const cd* st = nullptr;
  if (kLds) {
    cd* e = S + (size_t)(all_pairs ? max(b.n_pairs, 1) : 1) * n;
    st = e;
    const int u2 = b.Du * b.Du, v2 = b.Dv * b.Dv;
    for (int k = -1; k < b.n_pairs; ++k) {
      const cd* su = k < 0 ? b.Eu : b.Euk[k];
      const cd* sv = k < 0 ? b.Ev : b.Evk[k];
      for (int i = threadIdx.x; i < u2; i += kBlock) e[i] = su[i];
      for (int i = threadIdx.x; i < v2; i += kBlock) e[u2 + (i % b.Dv) * b.Dv + i / b.Dv] = sv[i];  // transposed
      e += u2 + v2;
    }
  }
  __shared__ double al[kMaxKrylov], be[kMaxKrylov];
  __shared__ cd hh[kRedStride];
  cd q = cz();
  for (int p = threadIdx.x; p < n; p += kBlock) q.x += cabs2(b.R[p]);
  q = block_sum(q, sm);
  const double nx = sqrt(q.x);
  if (nx == 0.0) return;
  const double inx = 1.0 / nx;
  for (int p = threadIdx.x; p < n; p += kBlock) V[p] = cscale(b.R[p], inx);
  __syncthreads();
  int k = 0;
  for (int j = 0; j < kmax; ++j) {
    bond_apply(b, st, V + (size_t)j * ld, W, S, all_pairs);
    double a_j = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      bond_dots(V, ld, W, n, j + 1, hh);
      for (int p = threadIdx.x; p < n; p += kBlock) {
        cd w = W[p];
        for (int i = 0; i <= j; ++i) {
          const cd h = hh[i];
          const cd v = V[(size_t)i * ld + p];
          w = csub(w, make_double2(h.x * v.x - h.y * v.y, h.x * v.y + h.y * v.x));
        }
        W[p] = w;
      }
      a_j += hh[j].x;
      __syncthreads();
    }
    cd nw = cz();
    for (int p = threadIdx.x; p < n; p += kBlock) nw.x += cabs2(W[p]);
    nw = block_sum(nw, sm);
    const double ww = sqrt(nw.x);
    if (threadIdx.x == 0) al[j] = a_j;
    k = j + 1;
    if (j == kmax - 1) break;
    if (ww <= tr.btol * nx) {
      if (threadIdx.x == 0) atomicAdd(&tr.stats[1], 1);
      break;
    }
    if (threadIdx.x == 0) be[j] = ww;
    const double iw = 1.0 / ww;
    for (int p = threadIdx.x; p < n; p += kBlock) V[(size_t)(j + 1) * ld + p] = cscale(W[p], iw);
    __syncthreads();
  }
  __syncthreads();
  krylov_exp(al, be, k, op.sign * (*T.half_step), sm);
  for (int p = threadIdx.x; p < n; p += kBlock) {
    cd acc = cz();
    for (int i = 0; i < k; ++i) acc = cfma(sm.vec[i], V[(size_t)i * ld + p], acc);
    b.R[p] = cscale(acc, nx);
  }
}

__device__ void body_bond(const Op& op, const DevTables& T, Smem& sm, cd* lds) {
  const TreeDev& tr = T.trees[op.tree];
  const BondDesc& b = T.bonds[op.desc];
  const int n = b.Du * b.Dv;
  const int kmax = min(tr.kmax, n);
  if (bond_lds_need(b, kmax, 1) <= (size_t)kQrLds) body_bond_t<true>(op, T, sm, lds);
  else body_bond_t<false>(op, T, sm, nullptr);
}

// ------------------------------------------------------------ fast bond step
// The bond step of body_bond_t (R <- exp(sign i h H_b) R by Lanczos with
// classical Gram-Schmidt applied twice, breakdown, Krylov dimension kmax)
// in one workgroup of kBondThreads threads with the Krylov basis, the work
// vectors and the environment matrices in LDS.
//   * H_b X = Eu X + X Ev^T + sum_k c_k Eu_k (X Ev_k^T): every thread owns
//     a 2 x 2 output block and a 1/S share of the summation index (S = 8, 4,
//     2 or 1, the most that keeps every block busy); the S partial blocks
//     of adjacent lanes are added by butterflies.  First Y (both products)
//     and every S_k = X Ev_k^T, then Y += sum_k c_k Eu_k S_k.
//   * the dot products V^H w use groups of L lanes per vector (as the fast
//     QR's projections), the second pass also carries |w|^2, and
//     beta = sqrt(|w1|^2 - |h2|^2) (the Pythagorean identity of the
//     projection); every thread keeps the residual of its elements in
//     registers.
constexpr int kBondThreads = 512;
constexpr int kBondRpt = 8;  // elements per thread (Du Dv <= 4096)

// one 2 x 2 block of sum_{m in [m0, m1)} A[a][m] B[m][c] (row-major, leading
// dimensions lda / ldb) added to y[4] (rows a0, a1; columns c0, c1)
__device__ __forceinline__ void bf_block(const cd* A, int lda, const cd* B, int ldb, int a0, int a1, int c0,
                                         int c1, int m0, int m1, cd* y) {
  for (int m = m0; m < m1; ++m) {
    const cd p0 = A[a0 * lda + m], p1 = A[a1 * lda + m];
    const cd q0 = B[m * ldb + c0], q1 = B[m * ldb + c1];
    y[0] = cfma(p0, q0, y[0]);
    y[1] = cfma(p0, q1, y[1]);
    y[2] = cfma(p1, q0, y[2]);
    y[3] = cfma(p1, q1, y[3]);
  }
}

template <int S>
__device__ __forceinline__ void bf_reduce(cd* y) {
#pragma unroll
  for (int off = S >> 1; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      y[q].x += __shfl_xor(y[q].x, off);
      y[q].y += __shfl_xor(y[q].y, off);
    }
}

// store (or with coef add coef *) a 2 x 2 block into Y (Du x Dv row-major)
__device__ __forceinline__ void bf_store(cd* Y, int Du, int Dv, int a0, int c0, const cd* y, bool add, double coef) {
  const int ia[4] = {a0, a0, a0 + 1, a0 + 1}, ic[4] = {c0, c0 + 1, c0, c0 + 1};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (ia[q] >= Du || ic[q] >= Dv) continue;
    cd* o = Y + ia[q] * Dv + ic[q];
    *o = add ? make_double2(fma(coef, y[q].x, o->x), fma(coef, y[q].y, o->y)) : y[q];
  }
}

// W = H_b X (st: Eu, Ev^T, then Eu_k, Ev_k^T per pair; Sb: n_pairs scratch
// matrices).  Ends with W visible to the workgroup.
template <int S>
__device__ void bf_apply(const BondDesc& b, const cd* st, const cd* X, cd* W, cd* Sb) {
  const int Du = b.Du, Dv = b.Dv, np = b.n_pairs;
  const int u2 = Du * Du, v2 = Dv * Dv;
  const int bu = (Du + 1) >> 1, bv = (Dv + 1) >> 1, nb = bu * bv;
  const int t = threadIdx.x;
  // phase A: item (product p, block, chunk); p = 0: Y = Eu X + X Ev^T,
  // p = 1 + k: S_k = X Ev_k^T
  const int itemsA = (1 + np) * nb * S;
  for (int base = 0; base < itemsA; base += kBondThreads) {  // uniform trip count
    const int it = base + t;
    const int ch = it % S, blk = (it / S) % nb, p = it / (S * nb);
    const int a0 = 2 * (blk / bv), c0 = 2 * (blk % bv);
    const int a1 = min(a0 + 1, Du - 1), c1 = min(c0 + 1, Dv - 1);
    cd y[4] = {cz(), cz(), cz(), cz()};
    if (it < itemsA) {
      const int v0 = ch * Dv / S, v1 = (ch + 1) * Dv / S;
      if (p == 0) {
        const int m0 = ch * Du / S, m1 = (ch + 1) * Du / S;
        bf_block(st, Du, X, Dv, a0, a1, c0, c1, m0, m1, y);           // Eu X
        bf_block(X, Dv, st + u2, Dv, a0, a1, c0, c1, v0, v1, y);      // X Ev^T
      } else {
        const cd* EvT = st + (size_t)p * (u2 + v2) + u2;
        bf_block(X, Dv, EvT, Dv, a0, a1, c0, c1, v0, v1, y);          // X Ev_k^T
      }
    }
    bf_reduce<S>(y);
    if (it < itemsA && ch == 0) bf_store(p == 0 ? W : Sb + (size_t)(p - 1) * Du * Dv, Du, Dv, a0, c0, y, false, 0.0);
  }
  lds_barrier();
  if (np == 0) return;
  // phase B: Y += sum_k c_k Eu_k S_k, item (block, chunk)
  const int itemsB = nb * S;
  for (int base = 0; base < itemsB; base += kBondThreads) {
    const int it = base + t;
    const int ch = it % S, blk = it / S;
    const int a0 = 2 * (blk / bv), c0 = 2 * (blk % bv);
    const int a1 = min(a0 + 1, Du - 1), c1 = min(c0 + 1, Dv - 1);
    const int m0 = ch * Du / S, m1 = (ch + 1) * Du / S;
    cd y[4] = {cz(), cz(), cz(), cz()};
    for (int k = 0; k < np; ++k) {
      cd z[4] = {cz(), cz(), cz(), cz()};
      if (it < itemsB) bf_block(st + (size_t)(k + 1) * (u2 + v2), Du, Sb + (size_t)k * Du * Dv, Dv, a0, a1, c0, c1, m0, m1, z);
      const double c = b.coef[k];
#pragma unroll
      for (int q = 0; q < 4; ++q) y[q] = make_double2(fma(c, z[q].x, y[q].x), fma(c, z[q].y, y[q].y));
    }
    bf_reduce<S>(y);
    if (it < itemsB && ch == 0) bf_store(W, Du, Dv, a0, c0, y, true, 1.0);
  }
  lds_barrier();
}

// h[i] = V_i^H x for i < cnt and, with `norm`, h[cnt] = |x|^2 (L lanes per
// entry, four chains each); ends with h visible.
template <int L>
__device__ void bf_dots(const cd* V, int n, const cd* x, int cnt, bool norm, cd* h) {
  const int t = threadIdx.x, i = t / L, g = t % L;
  const int ns = cnt + (norm ? 1 : 0);
  cd s0 = cz(), s1 = cz(), s2 = cz(), s3 = cz();
  if (i < cnt) {
    const cd* v = V + (size_t)i * n;
    int p = g;
    for (; p + 3 * L < n; p += 4 * L) {
      s0 = cjfma(v[p], x[p], s0);
      s1 = cjfma(v[p + L], x[p + L], s1);
      s2 = cjfma(v[p + 2 * L], x[p + 2 * L], s2);
      s3 = cjfma(v[p + 3 * L], x[p + 3 * L], s3);
    }
    for (; p < n; p += L) s0 = cjfma(v[p], x[p], s0);
  } else if (i == cnt && norm) {
    int p = g;
    for (; p + 3 * L < n; p += 4 * L) {
      s0.x += cabs2(x[p]);
      s1.x += cabs2(x[p + L]);
      s2.x += cabs2(x[p + 2 * L]);
      s3.x += cabs2(x[p + 3 * L]);
    }
    for (; p < n; p += L) s0.x += cabs2(x[p]);
  }
  cd s = cadd(cadd(s0, s1), cadd(s2, s3));
#pragma unroll
  for (int off = L >> 1; off > 0; off >>= 1) {
    s.x += __shfl_xor(s.x, off);
    s.y += __shfl_xor(s.y, off);
  }
  if (g == 0 && i < ns) h[i] = s;
  lds_barrier();
}
__device__ void bf_dots_any(const cd* V, int n, const cd* x, int cnt, bool norm, cd* h) {
  const int ns = cnt + (norm ? 1 : 0);
  if (ns <= kBondThreads / 64) bf_dots<64>(V, n, x, cnt, norm, h);
  else if (ns <= kBondThreads / 32) bf_dots<32>(V, n, x, cnt, norm, h);
  else bf_dots<16>(V, n, x, cnt, norm, h);  // ns <= kMaxKrylov + 1 < 32
}

// w - sum_{i<cnt} V_i[p] c[i], four chains
__device__ __forceinline__ cd bf_sub(const cd* V, int n, int p, int cnt, const cd* c, cd w) {
  cd w1 = cz(), w2 = cz(), w3 = cz();
  int i = 0;
  for (; i + 3 < cnt; i += 4) {
    const cd v0 = V[(size_t)i * n + p], v1 = V[(size_t)(i + 1) * n + p];
    const cd v2 = V[(size_t)(i + 2) * n + p], v3 = V[(size_t)(i + 3) * n + p];
    w = csub(w, make_double2(v0.x * c[i].x - v0.y * c[i].y, v0.x * c[i].y + v0.y * c[i].x));
    w1 = csub(w1, make_double2(v1.x * c[i + 1].x - v1.y * c[i + 1].y, v1.x * c[i + 1].y + v1.y * c[i + 1].x));
    w2 = csub(w2, make_double2(v2.x * c[i + 2].x - v2.y * c[i + 2].y, v2.x * c[i + 2].y + v2.y * c[i + 2].x));
    w3 = csub(w3, make_double2(v3.x * c[i + 3].x - v3.y * c[i + 3].y, v3.x * c[i + 3].y + v3.y * c[i + 3].x));
  }
  for (; i < cnt; ++i) {
    const cd v0 = V[(size_t)i * n + p];
    w = csub(w, make_double2(v0.x * c[i].x - v0.y * c[i].y, v0.x * c[i].y + v0.y * c[i].x));
  }
  return cadd(cadd(w, w1), cadd(w2, w3));
}

__global__ __launch_bounds__(kBondThreads) void k_bond_fast(Op op, DevTables T) {
  __shared__ __align__(16) cd lds[kBondFastLds];
  __shared__ Smem sm;  // Krylov exponential work (threads below kBlock)
  __shared__ double al[kMaxKrylov], be[kMaxKrylov], wsum[kBondThreads / 64];
  __shared__ cd h1[kMaxKrylov + 2], h2[kMaxKrylov + 2];
  const TreeDev& tr = T.trees[op.tree];
  const BondDesc& b = T.bonds[op.desc];
  const int Du = b.Du, Dv = b.Dv, n = Du * Dv, np = b.n_pairs;
  const int kmax = min(tr.kmax, n);
  const int t = threadIdx.x;
  cd* V = lds;                           // (kmax + 1) x n
  cd* W = V + (size_t)(kmax + 1) * n;    // n
  cd* Sb = W + n;                        // max(np, 1) x n
  cd* st = Sb + (size_t)max(np, 1) * n;  // Eu, Ev^T, then Eu_k, Ev_k^T per pair
  {
    const int u2 = Du * Du, v2 = Dv * Dv;
    cd* e = st;
    for (int k = -1; k < np; ++k) {
      const cd* su = k < 0 ? b.Eu : b.Euk[k];
      const cd* sv = k < 0 ? b.Ev : b.Evk[k];
      for (int i = t; i < u2; i += kBondThreads) e[i] = su[i];
      for (int i = t; i < v2; i += kBondThreads) e[u2 + (i % Dv) * Dv + i / Dv] = sv[i];  // transposed
      e += u2 + v2;
    }
  }
  // |R| and V_0 = R / |R|; every thread keeps its elements in registers
  cd w[kBondRpt];
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kBondRpt; ++q) {
    const int p = t + q * kBondThreads;
    w[q] = p < n ? b.R[p] : cz();
    s += cabs2(w[q]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((t & 63) == 0) wsum[t >> 6] = s;
  __syncthreads();  // also orders the staged matrices
  s = 0.0;
  for (int q = 0; q < kBondThreads / 64; ++q) s += wsum[q];
  const double nx = sqrt(s);
  if (nx == 0.0) return;  // uniform
  const double inx = 1.0 / nx;
#pragma unroll
  for (int q = 0; q < kBondRpt; ++q) {
    const int p = t + q * kBondThreads;
    if (p < n) V[p] = cscale(w[q], inx);
  }
  lds_barrier();
  const int bu = (Du + 1) >> 1, bv = (Dv + 1) >> 1, nb = bu * bv;
  const int S = nb * 8 <= kBondThreads ? 8 : nb * 4 <= kBondThreads ? 4 : nb * 2 <= kBondThreads ? 2 : 1;
  int k = 0;
  for (int j = 0; j < kmax; ++j) {
    const cd* vj = V + (size_t)j * n;
    switch (S) {
      case 8: bf_apply<8>(b, st, vj, W, Sb); break;
      case 4: bf_apply<4>(b, st, vj, W, Sb); break;
      case 2: bf_apply<2>(b, st, vj, W, Sb); break;
      default: bf_apply<1>(b, st, vj, W, Sb); break;
    }
    // first pass
    bf_dots_any(V, n, W, j + 1, false, h1);
#pragma unroll
    for (int q = 0; q < kBondRpt; ++q) {
      const int p = t + q * kBondThreads;
      if (p < n) w[q] = bf_sub(V, n, p, j + 1, h1, W[p]);
    }
    lds_barrier();  // W has been read
#pragma unroll
    for (int q = 0; q < kBondRpt; ++q) {
      const int p = t + q * kBondThreads;
      if (p < n) W[p] = w[q];
    }
    lds_barrier();
    // second pass with |w1|^2
    bf_dots_any(V, n, W, j + 1, true, h2);
    double hh = 0.0;
    for (int i = 0; i <= j; ++i) hh += cabs2(h2[i]);
    const double ww = sqrt(fmax(h2[j + 1].x - hh, 0.0));
    if (t == 0) al[j] = h1[j].x + h2[j].x;
    k = j + 1;
    if (j == kmax - 1) break;
    if (ww <= tr.btol * nx) {
      if (t == 0) atomicAdd(&tr.stats[1], 1);
      break;
    }
    if (t == 0) be[j] = ww;
    const double iw = 1.0 / ww;
    cd* vn = V + (size_t)(j + 1) * n;
#pragma unroll
    for (int q = 0; q < kBondRpt; ++q) {
      const int p = t + q * kBondThreads;
      if (p < n) vn[p] = cscale(bf_sub(V, n, p, j + 1, h2, w[q]), iw);
    }
    lds_barrier();
  }
  __syncthreads();  // al / be complete (krylov_exp reads them)
  krylov_exp(al, be, k, op.sign * (*T.half_step), sm);
#pragma unroll
  for (int q = 0; q < kBondRpt; ++q) {
    const int p = t + q * kBondThreads;
    if (p >= n) continue;
    cd acc = cz();
    for (int i = 0; i < k; ++i) acc = cfma(sm.vec[i], V[(size_t)i * n + p], acc);
    b.R[p] = cscale(acc, nx);
  }
}

// ------------------------------------------------------------ small ops
__device__ void body_copy(const Op& op, int vb) {
  const int idx = vb * kBlock + threadIdx.x;
  if (idx < op.n) op.p1[idx] = op.p0[idx];
}

// OP_DOT: Re <p0|p2> -> current record at double offset op.i1.
__device__ void body_dot(const Op& op, const DevTables& T, int vb, Smem& sm) {
  const TreeDev& tr = T.trees[op.tree];
  const int idx = vb * kBlock + threadIdx.x;
  cd p = cz();
  if (idx < op.n) p = cjfma(op.p0[idx], op.p2[idx], p);
  p = block_sum(p, sm);
  if (threadIdx.x == 0) tr.partials[vb * kRedStride] = p;
}
__device__ void fin_dot(const Op& op, const DevTables& T, int nvb, Smem& sm) {
  const TreeDev& tr = T.trees[op.tree];
  cd part = cz();
  for (int b = threadIdx.x; b < nvb; b += kBlock) part = cadd(part, tr.partials[b * kRedStride]);
  const double s = block_sum(part, sm).x;
  if (threadIdx.x == 0) {
    const int slot = min(*tr.rec_count, tr.rec_cap - 1);
    tr.hist[(size_t)slot * tr.rec_size + op.i1] = s;
  }
}

// OP_RECORD: norm = trace of the recorded density matrix (op.i0 levels,
// stored at offset 0, norm at offset op.i1); advance the record counter.
__device__ void body_record(const Op& op, const DevTables& T) {
  const TreeDev& tr = T.trees[op.tree];
  if (threadIdx.x == 0) {
    const int slot = min(*tr.rec_count, tr.rec_cap - 1);
    double* rec = tr.hist + (size_t)slot * tr.rec_size;
    double s = 0.0;
    for (int j = 0; j < op.i0; ++j) s += rec[2 * (j * op.i0 + j)];
    rec[op.i1] = s;
    if (!isfinite(s)) atomicOr(&tr.stats[3], 2);
    *tr.rec_count = min(*tr.rec_count + 1, tr.rec_cap);
    if (op.j) tr.stats[2] += 1;
  }
}

// ------------------------------------------------------------ executors
template <int TY>
__global__ __launch_bounds__(kBlock) void k_op(Op op, DevTables T) {
  __shared__ Smem sm;
  const int vb = blockIdx.x;
  if constexpr (TY == OP_SETH) {
    if (threadIdx.x == 0) *T.half_step = op.d0;
    return;
  }
  const TreeDev& tr = T.trees[op.tree];
  if constexpr (TY == OP_APPLY) {
    body_apply(op, T, vb);
  } else if constexpr (TY == OP_APPLY_LZ) {
    body_apply_lz(op, T, vb, sm);  // the next op folds the partial dots
  } else if constexpr (TY == OP_NORM) {
    body_norm(op, T, vb, sm);
    if (last_block(tr.counter, op.nvb, sm)) fin_norm(op, T, op.nvb, sm);
  } else if constexpr (TY == OP_SCALE) {
    body_scale(op, T, vb);
  } else if constexpr (TY == OP_ORTH1) {
    if (tr.scal->done) return;
    orth1_prologue(op, T, sm, vb == 0);
    body_orth1(op, T, vb, sm);
  } else if constexpr (TY == OP_ORTH2) {
    // fin_orth2 reads only values fixed before this launch (beta comes from
    // the norm identity of the first pass), so workgroup 0 can run it
    // without waiting for the others: no ticket
    if (tr.scal->done) return;
    orth2_prologue(op, sm);
    body_orth2(op, T, vb, sm);
    if (vb == 0) fin_orth2(op, T, sm);
  } else if constexpr (TY == OP_COMBINE) {
    body_combine(op, T, vb, sm);
  } else if constexpr (TY == OP_QR) {
    __shared__ cd qr_lds[kQrLds];
    body_qr<true>(op, T, sm, qr_lds);
  } else if constexpr (TY == OP_QRW) {
    if (body_qrw(op, T, vb, sm) && last_block(tr.counter, op.nvb, sm)) fin_qrw(op, T, op.nvb, sm);
  } else if constexpr (TY == OP_CONTRACT) {
    __shared__ cd ct_lds[2 * kCtRows * 64];
    body_contract(op, T, vb, sm, ct_lds);
    if (last_block(tr.counter, op.nvb, sm)) fin_contract(op, T, op.nvb);
  } else if constexpr (TY == OP_BOND) {
    __shared__ cd bond_lds[kQrLds];
    body_bond(op, T, sm, bond_lds);
  } else if constexpr (TY == OP_COPY) {
    body_copy(op, vb);
  } else if constexpr (TY == OP_DOT) {
    body_dot(op, T, vb, sm);
    if (last_block(tr.counter, op.nvb, sm)) fin_dot(op, T, op.nvb, sm);
  } else if constexpr (TY == OP_RECORD) {
    body_record(op, T);
  }
}

// One matrix-core group run by the calling workgroup, all its blocks in
// turn (the one-workgroup executor's form of the group kernel, with the
// same block code and so the same arithmetic): the reduced-precision forms
// only, with the small operand tile and 16 columns per block (the planner
// admits bonds up to 32 there), which keeps the executor's registers free
// of the larger tiles' accumulators.
__device__ void mode_group_in_workgroup(const Op& op, const DevTables& Tb, unsigned char* lds) {
  if (op.i0 == TTNS_FP32)
    mfma::mode_all_blocks<TTNS_FP32, mfma::Prec<TTNS_FP32>::SMALL, 16>(op, Tb, op.n, op.axis, lds);
  else if (op.i0 == TTNS_BF16X3)
    mfma::mode_all_blocks<TTNS_BF16X3, mfma::Prec<TTNS_BF16X3>::SMALL, 16>(op, Tb, op.n, op.axis, lds);
}
static_assert(mfma::ModeSmem<TTNS_FP32, mfma::Prec<TTNS_FP32>::SMALL, 16>::kBytes + 16 * 4 + 16 <= sizeof(cd) * kQrLds &&
                  mfma::ModeSmem<TTNS_BF16X3, mfma::Prec<TTNS_BF16X3>::SMALL, 16>::kBytes + 16 * 4 + 16 <=
                      sizeof(cd) * kQrLds,
              "matrix-core tiles exceed the executor's LDS");

// One workgroup runs the operation list of one tree: ops[begin[b], end[b]).
__global__ __launch_bounds__(kBlock) void k_persistent(const Op* __restrict__ ops,
                                                       const int* __restrict__ begin,
                                                       const int* __restrict__ end, DevTables T) {
  __shared__ Smem sm;
  __shared__ cd qr_lds[kQrLds];
  const int b = blockIdx.x;
  for (int i = begin[b]; i < end[b]; ++i) {
    const Op op = ops[i];
    const int nvb = op.nvb;
    switch (op.type) {
      case OP_APPLY:
        for (int vb = 0; vb < nvb; ++vb) body_apply(op, T, vb);
        break;
      case OP_APPLY_LZ: {
        bool act = true;
        for (int vb = 0; vb < nvb && act; ++vb) act = body_apply_lz(op, T, vb, sm);
        break;
      }
      case OP_NORM:
        for (int vb = 0; vb < nvb; ++vb) body_norm(op, T, vb, sm);
        __syncthreads();
        fin_norm(op, T, nvb, sm);
        break;
      case OP_SCALE:
        for (int vb = 0; vb < nvb; ++vb) body_scale(op, T, vb);
        break;
      case OP_ORTH1:
        if (T.trees[op.tree].scal->done) break;
        orth1_prologue(op, T, sm, true);
        for (int vb = 0; vb < nvb; ++vb) body_orth1(op, T, vb, sm);
        break;
      case OP_ORTH2:
        if (T.trees[op.tree].scal->done) break;
        orth2_prologue(op, sm);
        for (int vb = 0; vb < nvb; ++vb) body_orth2(op, T, vb, sm);
        __syncthreads();
        fin_orth2(op, T, sm);
        break;
      case OP_COMBINE:
        for (int vb = 0; vb < nvb; ++vb) body_combine(op, T, vb, sm);
        break;
      case OP_QR:
        body_qr<false>(op, T, sm, qr_lds);
        break;
      case OP_CONTRACT:
        for (int vb = 0; vb < nvb; ++vb) body_contract(op, T, vb, sm, qr_lds);
        __syncthreads();
        fin_contract(op, T, nvb);
        break;
      case OP_BOND:
        body_bond(op, T, sm, qr_lds);
        break;
      case OP_QRW: {
        bool act = false;
        for (int vb = 0; vb < nvb; ++vb) act = body_qrw(op, T, vb, sm) || act;
        __syncthreads();
        if (act) fin_qrw(op, T, nvb, sm);
        break;
      }
      case OP_COPY:
        for (int vb = 0; vb < nvb; ++vb) body_copy(op, vb);
        break;
      case OP_DOT:
        for (int vb = 0; vb < nvb; ++vb) body_dot(op, T, vb, sm);
        __syncthreads();
        fin_dot(op, T, nvb, sm);
        break;
      case OP_RECORD:
        body_record(op, T);
        break;
      case OP_MODE:
        mode_group_in_workgroup(op, T, reinterpret_cast<unsigned char*>(qr_lds));
        break;
      default:
        break;
    }
    __syncthreads();
  }
}

hipError_t launch_mode(const Op& op, const DevTables& t, hipStream_t s, int prec, int n_rest, int d);

hipError_t launch_op(const Op& op, const DevTables& t, hipStream_t s) {
  const dim3 grid(op.nvb > 0 ? op.nvb : 1), block(kBlock);
  if (op.type == OP_MODE) return launch_mode(op, t, s, op.i0, op.n, op.axis);
  if (op.type == OP_QR && op.i1 == 1) {
    hipLaunchKernelGGL(k_qr_fast, dim3(1), dim3(kQrThreads), 0, s, op, t);
    return hipGetLastError();
  }
  if (op.type == OP_BOND && op.i1 == 1) {
    hipLaunchKernelGGL(k_bond_fast, dim3(1), dim3(kBondThreads), 0, s, op, t);
    return hipGetLastError();
  }
  switch (op.type) {
#define TTNS_CASE(T_)                                            \
  case T_:                                                       \
    hipLaunchKernelGGL(k_op<T_>, grid, block, 0, s, op, t);      \
    break;
    TTNS_CASE(OP_APPLY)
    TTNS_CASE(OP_APPLY_LZ)
    TTNS_CASE(OP_NORM)
    TTNS_CASE(OP_SCALE)
    TTNS_CASE(OP_ORTH1)
    TTNS_CASE(OP_ORTH2)
    TTNS_CASE(OP_COMBINE)
    TTNS_CASE(OP_QR)
    TTNS_CASE(OP_CONTRACT)
    TTNS_CASE(OP_BOND)
    TTNS_CASE(OP_COPY)
    TTNS_CASE(OP_DOT)
    TTNS_CASE(OP_RECORD)
    TTNS_CASE(OP_SETH)
    TTNS_CASE(OP_QRW)
#undef TTNS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_persistent(const Op* dev_ops, const int* dev_begin, const int* dev_end,
                             int n_trees, const DevTables& t, hipStream_t s) {
  hipLaunchKernelGGL(k_persistent, dim3(n_trees), dim3(kBlock), 0, s, dev_ops, dev_begin,
                     dev_end, t);
  return hipGetLastError();
}

hipError_t launch_set_half_step(double* dst, double h, hipStream_t s) {
  Op op{};
  op.type = OP_SETH;
  op.nvb = 1;
  op.d0 = h;
  DevTables t{};
  t.half_step = dst;
  hipLaunchKernelGGL(k_op<OP_SETH>, dim3(1), dim3(kBlock), 0, s, op, t);
  return hipGetLastError();
}

}  // namespace ttns
