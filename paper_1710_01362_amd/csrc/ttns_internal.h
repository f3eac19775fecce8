// Internal types shared by the host planner (capi.cpp, model.cpp) and the
// device code (kernels.hip, mode_mfma.hip).  Plain structs of device pointers and sizes; the
// host builds tables of them once per context and the kernels read them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ttns.h"

namespace ttns {

constexpr int kMaxRank = 8;      // axes of a node tensor (parent, phys, children)
constexpr int kMaxEntries = 24;  // bond-channel terms in one H_eff apply
constexpr int kMaxTmp = 8;       // intermediate tensors for bond-bond terms
constexpr int kMaxKrylov = 16;   // Lanczos dimension limit
constexpr int kMaxPairs = 16;    // crossing terms on one bond
constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts)
constexpr int kRedStride = kMaxKrylov + 2;  // partial-sum slots per block
constexpr int kMaxQrVb = 64;     // workgroups of a wide QR
constexpr int kQrStride = 68;    // partial-sum slots per workgroup of a wide QR
constexpr int kQrLdsEntries = 8800;  // complex entries of the single-workgroup QR's LDS
constexpr int kQrThreads = 512;      // threads of the fast one-workgroup QR
constexpr int kQrRpt = 2;            // rows per thread of the fast QR
constexpr int kQrFastLds = 152 * 1024;  // LDS bytes of the fast QR
// LDS bytes the fast QR of a rows x cols matrix needs: Q, the residual
// vector, two coefficient vectors (+ norm slots), the column norms, and the
// span weight, tensor offset and completion-order entry of every row
constexpr size_t qr_fast_lds(int rows, int cols) {
  return (size_t)rows * cols * 16 + (size_t)rows * 16 + 2 * 66 * 16 + 64 * 16 + (size_t)rows * 14 + 64;
}
// complex entries of the fast bond step's LDS: Krylov basis, work vector,
// one scratch matrix per crossing term, the environment matrices
constexpr int kBondFastLds = 9216;
constexpr size_t bond_fast_lds(int Du, int Dv, int kmax, int pairs) {
  return (size_t)(kmax + 2 + (pairs > 1 ? pairs : 1)) * Du * Dv + (size_t)(1 + pairs) * (Du * Du + Dv * Dv);
}
constexpr bool bond_fast_fits(int Du, int Dv, int kmax, int pairs) {
  return Du * Dv <= 512 * 8 && bond_fast_lds(Du, Dv, kmax, pairs) <= (size_t)kBondFastLds;
}
constexpr bool qr_fast_fits(int rows, int cols) {
  return cols >= 1 && cols <= 63 && rows >= cols && rows <= kQrThreads * kQrRpt && rows <= 65535 &&
         qr_fast_lds(rows, cols) <= (size_t)kQrFastLds;
}

using cd = double2;  // complex double, interleaved (re, im)

// Row-major tensor shape of one node (axes: [parent], phys, children).
struct Shape {
  int rank;
  int phys_axis;
  int size;
  int dims[kMaxRank];
  int stride[kMaxRank];
};

// One term of an apply acting on a bond axis:
//   y += coef * op_phys o E_axis applied to src
// E is D x D row-major (E[a', a]); op is the physical operator (d x d,
// row-major) or null for the identity; [op_lo, op_hi] bounds the nonzero
// diagonals s' - s of op.  src = -1: the apply input x; else tmp[src].
struct Entry {
  int axis, src, op_lo, op_hi;
  double coef;
  const cd* E;
  const cd* op;
};

// y = site o x + sum_entries (...): an effective Hamiltonian (or a piece of
// one, or a single mode product) applied to one node tensor.
struct ApplyDesc {
  Shape sh;
  const cd* x;
  cd* y;
  const cd* tmp[kMaxTmp];
  const cd* site;  // summed on-site operator, or null
  double site_coef;
  int site_lo, site_hi;
  int n_entries;
  Entry e[kMaxEntries];
  double flops;  // algorithmic real flops of one apply (for reporting)
};

// One group of an H_eff apply on the matrix cores: every term acting on
// bond axis `axis` with the same source tensor,
//   y[s] (+)= sum_e E_e x_axis Z_{e,s},  Z_{e,s} = sum_o coef_e g_e(s, o) src[s + o],
// g_e(s, o) = op_e[s][s+o] (or delta_{o0}) over the band [lo_e, hi_e], with
// the complex products done as real GEMMs [[Re E, -Im E], [Im E, Re E]]
// . [Re Z; Im Z] on MFMA tiles (FP64, FP32 or split BF16).  The first group
// of an apply writes y (plus the on-site term), later ones add.
constexpr int kMaxGroup = 8;
struct ModeDesc {
  Shape sh;
  int axis;
  int prec;        // TTNS_FP64 / TTNS_FP32 / TTNS_BF16X3
  int accumulate;  // 0: y = site o x + group; 1: y += group
  int band_lo, band_hi;
  int n_rest;      // size / (dims[axis] * dims[phys])
  const cd* src;   // default source (x, or a temporary)
  const cd* x;     // apply input (for the on-site term)
  cd* y;
  const cd* site;
  double site_coef;
  int site_lo, site_hi;
  int n_e;
  const cd* E[kMaxGroup];
  const cd* op[kMaxGroup];
  int lo[kMaxGroup], hi[kMaxGroup];
  double coef[kMaxGroup];
  double flops;
};

// Bond effective Hamiltonian between u (rows of R) and v (columns):
//   H_b R = Eu R + R Ev^T + sum_k coef_k Eu_k R Ev_k^T
struct BondDesc {
  int Du, Dv;
  cd* R;
  const cd* Eu;
  const cd* Ev;
  int n_pairs;
  double coef[kMaxPairs];
  const cd* Euk[kMaxPairs];
  const cd* Evk[kMaxPairs];
};

// Scalars of the running Lanczos process of one tree.
struct LzScal {
  double nx, inv_nx;
  double alpha[kMaxKrylov];
  double beta[kMaxKrylov];
  cd h1[kRedStride];
  cd h2[kRedStride];
  double ww1, ww2;
  int k_eff, done;
  int pad[2];
};

// Scalars of a running wide (multi-workgroup) QR.
struct QrScal {
  double tol, rn, iu;
  int deficient, row;
  cd h1[64], h2[64];
};

// Per-tree device scratch (all inside the caller's workspace).
struct TreeDev {
  LzScal* scal;
  cd* V;            // (kmax + 1) x ldv Krylov basis
  cd* W;            // ldv
  cd* Z;            // ldv: environment / observable intermediates
  cd* X;            // ldv: absorb target before it is copied back
  cd* tmp[kMaxTmp]; // ldv each
  cd* R;            // bond matrix, maxD^2
  cd* bondV;        // (kmax + 1) x maxD^2
  cd* bondW;        // 3 x maxD^2
  cd* qrA;          // ldv (column-major matricisation)
  cd* qrQ;          // ldv
  cd* qrv;          // 2 x maxrows residual / completion vectors
  cd* partials;     // max_nvb x kRedStride
  cd* cpart;        // contraction partial matrices, max_nvb x maxD^2
  cd* qrpart;       // wide-QR partial sums, kMaxQrVb x kQrStride
  QrScal* qrs;
  unsigned* counter;
  double* hist;     // rec_cap x rec_size
  int* rec_count;
  int* stats;       // [0] guarded columns, [1] breakdowns, [2] steps
  int ldv;
  int max_rows;
  int rec_size, rec_cap;
  int kmax;
  double btol, rtol;
};

enum OpType : int {
  OP_APPLY = 0,   // desc: y = H x
  OP_APPLY_LZ,    // desc with x := V_j, y := W, plus dots with V_0..V_j
  OP_NORM,        // |x| -> scal (starts a Lanczos process)
  OP_SCALE,       // V_0 = x / |x|
  OP_ORTH1,       // first Gram-Schmidt pass
  OP_ORTH2,       // second pass, beta_j, V_{j+1}
  OP_COMBINE,     // out = |x| V exp(sign*i*h*T) e_1
  OP_QR,          // guarded QR of a node tensor towards an axis
  OP_CONTRACT,    // E = Q_(axis)^H Z_(axis)
  OP_BOND,        // whole bond exponential (one workgroup)
  OP_COPY,        // dst = src
  OP_DOT,         // <a|b> into the record
  OP_RECORD,      // close the record of this step
  OP_SETH,        // set the half step of the context
  OP_QRW,         // one phase of a wide QR (op.i0 = phase, op.j = column)
  OP_MODE,        // one MFMA group of an apply (ModeDesc op.desc; p0/p1 override src/y)
  OP_COUNT
};

// One step of a tree program.  Field use per type is documented at the
// device implementation of each op.
struct Op {
  int type;
  int nvb;    // virtual workgroups
  int tree;   // index into the TreeDev table
  int desc;   // ApplyDesc / BondDesc index, or -1
  int j;      // Lanczos index
  int sign;   // exponent sign (-1 node, +1 bond)
  int n;      // element count
  int axis;
  int i0, i1; // op-specific integers
  const cd* p0;
  cd* p1;
  const cd* p2;
  double d0;
};

// ---------------------------------------------------------------- host side

struct HostTerm {
  int a, opa, b, opb;  // b = -1 on-site
  double coef;
};

struct HostTree {
  int n = 0;
  std::vector<int> parent, phys, bondreq;
  std::vector<std::vector<cd>> ops;
  std::vector<int> opdim;
  std::vector<HostTerm> terms;
  std::vector<std::vector<cd>> init;
  std::vector<int> obs_node, obs_op;
  int n_levels_hint = 0;  // for star models: electronic levels at the root
};

// model.cpp
bool star_to_tree(const ttns_star_model& m, HostTree& t, std::string& err);
bool api_to_tree(const ttns_tree& a, HostTree& t, std::string& err);

// kernels.hip: device entry points used by the executors
struct DevTables {
  const ApplyDesc* descs;
  const ModeDesc* modes;
  const BondDesc* bonds;
  const TreeDev* trees;
  double* half_step;  // context-wide h = dt / 2
};

hipError_t launch_op(const Op& op, const DevTables& t, hipStream_t s);
hipError_t launch_persistent(const Op* dev_ops, const int* dev_begin,
                             const int* dev_end, int n_trees,
                             const DevTables& t, hipStream_t s);
hipError_t launch_set_half_step(double* dst, double h, hipStream_t s);

// surfaces.hip: dense kernels of the energy surfaces and bond entropy
int surf_eig_max();
hipError_t launch_herm_eig(const cd* A, int N, int lda, double* evals, cd* vecs, int graded, hipStream_t s);
hipError_t launch_bath_vectors(const cd* X, int ldx, int nel, int nb, const cd* W, const double* lam, int r,
                               int normalise, cd* B, int ldb, hipStream_t s);
hipError_t launch_surf_fill(cd* X, const cd* B, int ldb, int k, int l, int nel, int nb, hipStream_t s);
hipError_t launch_surf_dots(const cd* B, int ldb, const cd* Y, int ldy, int nel, int nb, int r, cd* part, int nvb,
                            hipStream_t s);
hipError_t launch_surf_fold(const cd* part, int nvb, int cnt, cd* M, int ldm, int col, hipStream_t s);
hipError_t launch_gram(const cd* R, int D, cd* G, hipStream_t s);
hipError_t launch_entropy(const double* lam, int N, double* out, hipStream_t s);

// MFMA limits: largest bond dimension per precision
int mode_max_bond(int prec);
// padded real operand size (2D rounded up to the MFMA K granule) of a group
int mode_padded(int prec, int D);
// largest padded size the small matrix-core tile takes
int mode_small_dp(int prec);
// default column tile: 16 columns when 64-column tiles give too few workgroups
bool mode_default_narrow(int n_rest, int d);

}  // namespace ttns
