// Small dense kernels of the energy surfaces (Eqs. 3-4) and the bond
// entanglement entropy: a one-workgroup Hermitian eigensolver (cyclic
// Jacobi with complex rotations, disjoint pairs rotated together), the bath
// Schmidt states of the root, the projected matrix of an effective
// Hamiltonian between (bath state, electronic state) products, and the
// entropy of a bond matrix's Schmidt values.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "ttns_internal.h"

namespace ttns {

namespace {

constexpr int kEigMax = 64;   // largest matrix of the eigensolver
constexpr int kEigSweeps = 60;

// Eigenvalues (ascending, evals[0..N)) and, with vecs, eigenvectors (column
// j of vecs[r * N + j], row-major) of the Hermitian part (A + A^H) / 2 of
// the N x N matrix A (row-major, leading dimension lda).  Sweeps end when
// the off-diagonal weight is below 1e-30 of the total and, with `graded`
// (a positive semi-definite matrix whose diagonal spans many orders, such
// as a Gram matrix of nearly orthogonal rows), also every |a_pq|^2 is below
// 1e-30 a_pp a_qq, which keeps the small eigenvalues' vectors accurate to
// rounding relative to their own size.
__global__ __launch_bounds__(kBlock) void k_herm_eig(const cd* __restrict__ Ain, int N, int lda,
                                                     double* evals, cd* vecs, int graded) {
  __shared__ cd A[kEigMax * kEigMax];
  __shared__ cd V[kEigMax * kEigMax];
  __shared__ double rc[kEigMax / 2], rs[kEigMax / 2];
  __shared__ cd rph[kEigMax / 2];
  __shared__ int pp[kEigMax / 2], pq[kEigMax / 2];
  __shared__ double red[kBlock / 64][3];
  __shared__ int order[kEigMax];
  const int t = threadIdx.x;
  for (int i = t; i < N * N; i += kBlock) {
    const int r = i / N, c = i % N;
    const cd a = Ain[r * lda + c], b = Ain[c * lda + r];
    A[i] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    V[i] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int Np = (N + 1) & ~1;  // players of the round-robin (one idle when N is odd)
  const int half = Np / 2;
  for (int sweep = 0; sweep < kEigSweeps; ++sweep) {
    // convergence: off-diagonal weight against the total
    double off = 0.0, tot = 0.0, rel = 0.0;
    for (int i = t; i < N * N; i += kBlock) {
      const int r = i / N, c = i % N;
      const double w = cabs2(A[i]);
      tot += w;
      if (r != c) {
        off += w;
        const double dd = A[r * N + r].x * A[c * N + c].x;
        if (graded && w > 0.0) rel = fmax(rel, dd > 0.0 ? w / dd : 1.0);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      tot += __shfl_xor(tot, o);
      rel = fmax(rel, __shfl_xor(rel, o));
    }
    if ((t & 63) == 0) {
      red[t >> 6][0] = off;
      red[t >> 6][1] = tot;
      red[t >> 6][2] = rel;
    }
    __syncthreads();
    off = tot = rel = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      off += red[w][0];
      tot += red[w][1];
      rel = fmax(rel, red[w][2]);
    }
    __syncthreads();
    // uniform (also ends on tot = 0 or NaN)
    if (!(off > 1e-30 * tot) && !(rel > 1e-30)) break;
    for (int round = 0; round < Np - 1; ++round) {
      // pairs of this round: player 0 fixed, the others rotate
      if (t < half) {
        auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (Np - 1); };
        int p = player(t), q = player(Np - 1 - t);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        double c = 1.0, s = 0.0;
        cd ph = make_double2(1.0, 0.0);
        if (q < N) {
          const cd apq = A[p * N + q];
          const double m = sqrt(cabs2(apq));
          if (m > 1e-300) {
            const double tau = (A[q * N + q].x - A[p * N + p].x) / (2.0 * m);
            const double tn = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tn * tn);
            s = tn * c;
            ph = make_double2(apq.x / m, -apq.y / m);  // e^{-i phi}, apq = m e^{i phi}
          }
        }
        pp[t] = p;
        pq[t] = q;
        rc[t] = c;
        rs[t] = s;
        rph[t] = ph;
      }
      __syncthreads();
      // A <- A J, V <- V J with J_pp = c, J_pq = s, J_qp = -s e^{-i phi},
      // J_qq = c e^{-i phi} (columns p, q of every pair)
      for (int i = t; i < half * N; i += kBlock) {
        const int k = i / N, r = i % N;
        const int p = pp[k], q = pq[k];
        if (q >= N) continue;
        const double c = rc[k], s = rs[k];
        const cd ph = rph[k];
        const cd x = A[r * N + p], y = A[r * N + q];
        const cd yph = make_double2(y.x * ph.x - y.y * ph.y, y.x * ph.y + y.y * ph.x);
        A[r * N + p] = make_double2(c * x.x - s * yph.x, c * x.y - s * yph.y);
        A[r * N + q] = make_double2(s * x.x + c * yph.x, s * x.y + c * yph.y);
        const cd vx = V[r * N + p], vy = V[r * N + q];
        const cd vph = make_double2(vy.x * ph.x - vy.y * ph.y, vy.x * ph.y + vy.y * ph.x);
        V[r * N + p] = make_double2(c * vx.x - s * vph.x, c * vx.y - s * vph.y);
        V[r * N + q] = make_double2(s * vx.x + c * vph.x, s * vx.y + c * vph.y);
      }
      __syncthreads();
      // A <- J^H A (rows p, q of every pair)
      for (int i = t; i < half * N; i += kBlock) {
        const int k = i / N, col = i % N;
        const int p = pp[k], q = pq[k];
        if (q >= N) continue;
        const double c = rc[k], s = rs[k];
        const cd phc = make_double2(rph[k].x, -rph[k].y);  // e^{+i phi}
        const cd x = A[p * N + col], y = A[q * N + col];
        const cd yph = make_double2(y.x * phc.x - y.y * phc.y, y.x * phc.y + y.y * phc.x);
        A[p * N + col] = make_double2(c * x.x - s * yph.x, c * x.y - s * yph.y);
        A[q * N + col] = make_double2(s * x.x + c * yph.x, s * x.y + c * yph.y);
      }
      __syncthreads();
    }
  }
  // ascending order of the diagonal (stable selection by rank)
  for (int i = t; i < N; i += kBlock) {
    const double di = A[i * N + i].x;
    int rank = 0;
    for (int j = 0; j < N; ++j) {
      const double dj = A[j * N + j].x;
      rank += (dj < di) || (dj == di && j < i);
    }
    order[rank] = i;
  }
  __syncthreads();
  for (int i = t; i < N; i += kBlock) evals[i] = A[order[i] * N + order[i]].x;
  if (vecs)
    for (int i = t; i < N * N; i += kBlock) {
      const int r = i / N, j = i % N;
      vecs[r * N + j] = V[r * N + order[j]];
    }
}

// Rows of the nel x nb matrix X (leading dimension ldx) rotated by the
// eigenvectors W of G = conj(X X^H) (ascending eigenvalues lam): output row
// i (i < r) is sum_m W[m, nel-1-i] X[m, :], divided by sqrt(lam[nel-1-i])
// when `normalise`.  (W's columns are the conjugates of X X^H's
// eigenvectors u, so sum_m conj(u[m]) X[m, :] = u^H X needs no conjugate.)
__global__ __launch_bounds__(kBlock) void k_bath_vectors(const cd* __restrict__ X, int ldx, int nel, int nb,
                                                         const cd* __restrict__ W, const double* lam, int r,
                                                         int normalise, cd* B, int ldb) {
  const int beta = blockIdx.x * kBlock + threadIdx.x;
  if (beta >= nb) return;
  for (int i = 0; i < r; ++i) {
    const int col = nel - 1 - i;
    cd acc = cz();
    for (int m = 0; m < nel; ++m) acc = cfma(W[m * nel + col], X[(size_t)m * ldx + beta], acc);
    B[(size_t)i * ldb + beta] = normalise ? cscale(acc, 1.0 / sqrt(lam[col])) : acc;
  }
}

// X[sigma, beta] = delta(sigma, l) B[k, beta]
__global__ __launch_bounds__(kBlock) void k_surf_fill(cd* X, const cd* __restrict__ B, int ldb, int k, int l,
                                                      int nel, int nb) {
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= nel * nb) return;
  const int sg = idx / nb, beta = idx - sg * nb;
  X[idx] = sg == l ? B[(size_t)k * ldb + beta] : cz();
}

// part[vb * cnt + (i * nel + j)] = sum over this block's betas of
// conj(B[i, beta]) Y[j, beta]  (rows of Y at stride ldy; cnt = r * nel <=
// kEigMax)
__global__ __launch_bounds__(kBlock) void k_surf_dots(const cd* __restrict__ B, int ldb, const cd* __restrict__ Y,
                                                      int ldy, int nel, int nb, int r, cd* part) {
  __shared__ cd wsum[kBlock / 64][kEigMax];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int chunk = (nb + gridDim.x - 1) / gridDim.x;
  const int b0 = blockIdx.x * chunk, b1 = min(nb, b0 + chunk);
  const int cnt = r * nel;
  for (int a = 0; a < cnt; ++a) {
    const int i = a / nel, j = a % nel;
    cd s = cz();
    for (int beta = b0 + t; beta < b1; beta += kBlock) s = cjfma(B[(size_t)i * ldb + beta], Y[(size_t)j * ldy + beta], s);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      s.x += __shfl_xor(s.x, o);
      s.y += __shfl_xor(s.y, o);
    }
    if (lane == 0) wsum[wid][a] = s;
  }
  __syncthreads();
  for (int a = t; a < cnt; a += kBlock) {
    cd s = wsum[0][a];
    for (int w = 1; w < kBlock / 64; ++w) s = cadd(s, wsum[w][a]);
    part[(size_t)blockIdx.x * cnt + a] = s;
  }
}

// M[a * ldm + col] = sum_vb part[vb * cnt + a]   (blocks in order)
__global__ __launch_bounds__(kBlock) void k_surf_fold(const cd* __restrict__ part, int nvb, int cnt, cd* M,
                                                      int ldm, int col) {
  const int a = threadIdx.x;
  if (a >= cnt) return;
  cd s = cz();
  for (int b = 0; b < nvb; ++b) s = cadd(s, part[(size_t)b * cnt + a]);
  M[(size_t)a * ldm + col] = s;
}

// G = R^H R for the D x D bond matrix R (row-major)
__global__ __launch_bounds__(kBlock) void k_gram(const cd* __restrict__ R, int D, cd* G) {
  for (int p = threadIdx.x; p < D * D; p += kBlock) {
    const int i = p / D, j = p % D;
    cd s = cz();
    for (int k = 0; k < D; ++k) s = cjfma(R[k * D + i], R[k * D + j], s);
    G[p] = s;
  }
}

// -sum p ln p over p = lam / sum(lam) (negative rounding of lam clipped)
__global__ void k_entropy(const double* lam, int N, double* out) {
  if (threadIdx.x != 0) return;
  double sum = 0.0;
  for (int i = 0; i < N; ++i) sum += fmax(lam[i], 0.0);
  double S = 0.0;
  if (sum > 0.0)
    for (int i = 0; i < N; ++i) {
      const double p = fmax(lam[i], 0.0) / sum;
      if (p > 1e-300) S -= p * log(p);
    }
  *out = S;
}

}  // namespace

int surf_eig_max() { return kEigMax; }

hipError_t launch_herm_eig(const cd* A, int N, int lda, double* evals, cd* vecs, int graded, hipStream_t s) {
  if (N < 1 || N > kEigMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_herm_eig, dim3(1), dim3(kBlock), 0, s, A, N, lda, evals, vecs, graded);
  return hipGetLastError();
}
hipError_t launch_bath_vectors(const cd* X, int ldx, int nel, int nb, const cd* W, const double* lam, int r,
                               int normalise, cd* B, int ldb, hipStream_t s) {
  hipLaunchKernelGGL(k_bath_vectors, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, s, X, ldx, nel, nb, W, lam,
                     r, normalise, B, ldb);
  return hipGetLastError();
}
hipError_t launch_surf_fill(cd* X, const cd* B, int ldb, int k, int l, int nel, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_surf_fill, dim3((nel * nb + kBlock - 1) / kBlock), dim3(kBlock), 0, s, X, B, ldb, k, l, nel,
                     nb);
  return hipGetLastError();
}
hipError_t launch_surf_dots(const cd* B, int ldb, const cd* Y, int ldy, int nel, int nb, int r, cd* part, int nvb,
                            hipStream_t s) {
  if (r * nel > kEigMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_surf_dots, dim3(nvb), dim3(kBlock), 0, s, B, ldb, Y, ldy, nel, nb, r, part);
  return hipGetLastError();
}
hipError_t launch_surf_fold(const cd* part, int nvb, int cnt, cd* M, int ldm, int col, hipStream_t s) {
  hipLaunchKernelGGL(k_surf_fold, dim3(1), dim3(kBlock), 0, s, part, nvb, cnt, M, ldm, col);
  return hipGetLastError();
}
hipError_t launch_gram(const cd* R, int D, cd* G, hipStream_t s) {
  hipLaunchKernelGGL(k_gram, dim3(1), dim3(kBlock), 0, s, R, D, G);
  return hipGetLastError();
}
hipError_t launch_entropy(const double* lam, int N, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_entropy, dim3(1), dim3(64), 0, s, lam, N, out);
  return hipGetLastError();
}

}  // namespace ttns
