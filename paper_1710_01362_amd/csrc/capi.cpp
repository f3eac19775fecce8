// Host side of the TTNS library: validation, channel analysis, workspace
// layout, the operation programs of the one-site TDVP step, the executors
// (wide kernels captured in a HIP graph, or one persistent workgroup per
// tree) and the C-ABI entry points of include/ttns.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ttns_internal.h"
#include "../../include/ttnn.h"

namespace ttns {
void ohmic_chain(double alpha, double wc, double s, int L, double* c0, double* eps, double* hop);
}

using namespace ttns;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return fail(TTNS_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int PHYS = -1;
constexpr int kMaxD = 64;       // QR keeps per-column scalars in shared arrays
constexpr int kMaxContractVb = 64;
constexpr int kMfmaMinSize = 16384;  // nodes this large use the matrix cores
constexpr size_t kGraphSegment = 8192;  // launches per captured graph
constexpr int kQrOneGroupRows = 4096;   // tallest QR left to one workgroup
constexpr int kSplitLanes = 65536;      // scalar applies spread small nodes over up to this many lanes
constexpr int kSurfVb = 256;            // workgroups of the energy-surface projections
constexpr int kAuxMat = 64 * 64;        // entries of one eigensolver matrix
// context-wide scratch: matrix, eigenvectors, eigenvalues (+ one result
// double), projection partial sums
size_t aux_bytes() { return 2 * kAuxMat * sizeof(cd) + 256 * sizeof(double) + (size_t)kSurfVb * 64 * sizeof(cd); }

// Channel of an environment: the block Hamiltonian (kind 0), one end of a
// two-node term (kind 1: term k, end 0 = node_a / 1 = node_b) or a recorded
// local observable (kind 2: observable k).
struct ChanKey {
  int kind, k, end;
  bool operator==(const ChanKey& o) const { return kind == o.kind && k == o.k && end == o.end; }
};

struct Env {
  std::vector<ChanKey> keys;
  size_t off = 0;  // byte offset in the workspace
  cd* base = nullptr;
  int D = 0;
  cd* chan(const ChanKey& key) const {
    for (size_t i = 0; i < keys.size(); ++i)
      if (keys[i] == key) return base + i * (size_t)D * D;
    return nullptr;
  }
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct TreeState {
  HostTree ht;
  int n = 0;
  std::vector<std::vector<int>> children;
  std::vector<int> sub, D;
  std::vector<Shape> shape;
  std::map<std::pair<int, int>, Env> env;
  std::vector<int> op_lo, op_hi;
  std::vector<std::vector<cd>> site;  // summed on-site operator per node (empty: none)
  std::vector<int> site_lo, site_hi;
  int maxsize = 1, maxD = 1, max_rows = 1, ntmp = 0, max_nvb = 1;
  int maxC = 1;  // largest contraction dimension (bonds and the root's levels)
  int n_el = 1, rec_size = 0, kmax = 12;
  // workspace offsets (bytes)
  size_t o_scal, o_counter, o_rec, o_stats, o_V, o_W, o_Z, o_X, o_tmp, o_R, o_bondV, o_bondW,
      o_qrA, o_qrQ, o_qrv, o_part, o_cpart, o_hist, o_ops, o_site, o_qrpart, o_qrs;
  std::vector<size_t> o_T, o_opdata, o_sitedata;
  // device pointers
  std::vector<cd*> T, opdev, sitedev;
  TreeDev dev{};
  int centre = 0;
  std::vector<int> heff_desc;                 // H_eff of every node (x = T_v, y = W)
  std::vector<std::vector<int>> heff_pre;     // its bond-bond pre-stages
  struct EdgePlan {
    std::vector<int> chan_desc;               // one per environment channel
    std::vector<int> h_pre;                   // pre-stages of the H channel
    int absorb_desc = -1;                     // R into the far node
    int bond_desc = -1;
  };
  std::map<std::pair<int, int>, EdgePlan> edge;  // directed edge (u -> w)
  std::vector<int> obs_desc;                  // recorded observables at the root
  // H_eff on the matrix cores (empty: the node uses the scalar apply)
  std::vector<std::vector<int>> mode_pre;     // bond-bond pre-stages (ModeDesc ids)
  std::vector<std::vector<int>> mode_groups;  // groups; the first carries the site term
  std::vector<int> mode_tile;                 // 0 default, else the autotuner's tile (op.i1 code:
                                              // 1 small / 2 large operands, + 4 for 16 columns)
};

bool in_subtree(const TreeState& t, int node, int v) { return node >= v && node < v + t.sub[v]; }
int parent_of(const TreeState& t, int v) { return t.ht.parent[v]; }

// is `node` on u's side of the edge (u, v)?
bool in_side(const TreeState& t, int node, int u, int v) {
  if (u != 0 && v == parent_of(t, u)) return in_subtree(t, node, u);
  return !in_subtree(t, node, v);
}

int region(const TreeState& t, int v, int node) {
  if (node == v) return PHYS;
  if (in_subtree(t, node, v)) {
    for (int c : t.children[v])
      if (in_subtree(t, node, c)) return c;
  }
  return parent_of(t, v);
}

int axis_of(const TreeState& t, int v, int u) {
  const int pa = v == 0 ? 0 : 1;
  if (u == PHYS) return pa;
  if (v != 0 && u == parent_of(t, v)) return 0;
  const auto& ch = t.children[v];
  for (size_t i = 0; i < ch.size(); ++i)
    if (ch[i] == u) return pa + 1 + (int)i;
  return -1;
}

std::vector<int> nbrs(const TreeState& t, int v) {
  std::vector<int> r;
  if (v != 0) r.push_back(parent_of(t, v));
  for (int c : t.children[v]) r.push_back(c);
  return r;
}

void band_of(const std::vector<cd>& m, int d, int& lo, int& hi) {
  lo = d;
  hi = -d;
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c)
      if (m[r * d + c].x != 0.0 || m[r * d + c].y != 0.0) {
        lo = std::min(lo, c - r);
        hi = std::max(hi, c - r);
      }
  if (lo > hi) lo = hi = 0;
}

// trace(A^op1 B^op2) helpers for the Hermiticity check
cd tr_prod(const std::vector<cd>& A, bool adjA, const std::vector<cd>& B, bool adjB, int d) {
  cd s{0, 0};
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      cd a = adjA ? cd{A[j * d + i].x, -A[j * d + i].y} : A[i * d + j];
      cd b = adjB ? cd{B[i * d + j].x, -B[i * d + j].y} : B[j * d + i];
      s.x += a.x * b.x - a.y * b.y;
      s.y += a.x * b.y + a.y * b.x;
    }
  return s;
}
cd cmulh(cd a, cd b) { return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// |sum_k c_k (A_k (x) B_k - A_k^+ (x) B_k^+)|_F^2 via traces of d x d products.
double herm_defect(const TreeState& t, const std::vector<int>& ks, bool onsite) {
  double tot = 0.0;
  const auto& H = t.ht;
  for (int k : ks)
    for (int l : ks) {
      const HostTerm &a = H.terms[k], &b = H.terms[l];
      const int da = H.opdim[a.opa];
      // (X_k)^+ X_l with X = A(x)B - A^+(x)B^+ ; tr over the product space factorises
      auto term = [&](bool k1, bool l1) -> cd {  // k1/l1: adjoint taken in X_k / X_l part
        cd ta = tr_prod(H.ops[a.opa], !k1, H.ops[b.opa], l1, da);
        if (onsite) return ta;
        const int db = H.opdim[a.opb];
        cd tb = tr_prod(H.ops[a.opb], !k1, H.ops[b.opb], l1, db);
        return cmulh(ta, tb);
      };
      // X_k^+ X_l = (A^+ (x) B^+ - A (x) B)(A_l (x) B_l - A_l^+ (x) B_l^+)
      cd s = term(false, false);
      cd s2 = term(false, true);
      cd s3 = term(true, false);
      cd s4 = term(true, true);
      tot += a.coef * b.coef * (s.x - s2.x - s3.x + s4.x);
    }
  return tot;
}

}  // namespace

struct ttns_ctx {
  ttns_opts opts{};
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<TreeState> trees;
  std::vector<ApplyDesc> descs;
  std::vector<BondDesc> bonds;
  std::vector<ModeDesc> modes;
  size_t o_modes = 0;
  size_t o_aux = 0;  // context-wide scratch of the energy surfaces and bond entropy
  size_t o_descs = 0, o_bonds = 0, o_trees = 0, o_half = 0, o_prog = 0, o_begin = 0, o_end = 0;
  size_t total = 0;
  DevTables tables{};
  Op* d_ops = nullptr;
  int* d_begin = nullptr;
  int* d_end = nullptr;
  std::vector<Op> step_ops;        // wide program of one step (all trees)
  std::vector<int> tree_begin, tree_end;
  std::vector<Op> tree_prog;       // persistent program (per tree contiguous)
  // one step as a sequence of captured graphs of at most kGraphSegment
  // launches each (instantiation cost and host memory grow with the node
  // count; a large tree's step holds hundreds of thousands of launches)
  std::vector<hipGraph_t> graphs;
  std::vector<hipGraphExec_t> gexecs;
  bool persistent = false;
  bool profile = false;
  double prof_ms = 0.0, prof_flops = 0.0;
  int64_t prof_n = 0;
  struct Pending {
    hipEvent_t e0, e1;
    int cls;
    double flops, bytes;
  };
  std::vector<Pending> ev_pool;
  double cls_ms[TTNS_K_COUNT] = {0}, cls_flops[TTNS_K_COUNT] = {0}, cls_bytes[TTNS_K_COUNT] = {0};
  int64_t cls_n[TTNS_K_COUNT] = {0};
  double last_h = -1e300;
  int scratch_desc = 0;  // first of the descriptor slots ttns_apply_heff rewrites
  std::vector<double> step_flops, heff_flops;  // per tree, algorithmic
  // autotuner: the probe build plans every candidate; the final build
  // follows the measured choices
  bool tune_probe = false;
  std::map<std::string, int> tune_heff;  // node class -> 0 scalar, else the matrix-core tile (op.i1 code)
  std::map<std::string, int> tune_qr;    // QR shape -> 0 one workgroup, k > 0 wide with k workgroups
  std::string tune_report;
  std::string err;  // message of the last failed call on this context
  // built by ttns_star_build_noalloc: the workspace is this device's static
  // array, steps run launch by launch (no capture stream, no graphs)
  bool noalloc = false;
  int noalloc_dev = -1;
};

namespace {

// ------------------------------------------------------------------ analysis
int analyze(TreeState& t, const ttns_opts& o, std::string& err) {
  HostTree& H = t.ht;
  t.n = H.n;
  const int n = t.n;
  if (n < 1 || (int)H.parent.size() != n || H.parent[0] != -1) {
    err = "tree: parent[0] must be -1";
    return TTNS_EINVAL;
  }
  t.children.assign(n, {});
  for (int v = 1; v < n; ++v) {
    if (H.parent[v] < 0 || H.parent[v] >= v) {
      err = "tree: parent[i] must lie in [0, i)";
      return TTNS_EINVAL;
    }
    t.children[H.parent[v]].push_back(v);
  }
  t.sub.assign(n, 1);
  for (int v = n - 1; v > 0; --v) t.sub[H.parent[v]] += t.sub[v];
  for (int v = 0; v < n; ++v) {  // pre-order: children follow their parent contiguously
    int next = v + 1;
    for (int c : t.children[v]) {
      if (c != next) {
        err = "tree: nodes must be numbered in pre-order";
        return TTNS_EINVAL;
      }
      next = c + t.sub[c];
    }
  }
  for (size_t k = 0; k < H.ops.size(); ++k)
    if ((int)H.ops[k].size() != H.opdim[k] * H.opdim[k]) {
      err = "tree: operator data size";
      return TTNS_EINVAL;
    }
  for (const HostTerm& x : H.terms) {
    if (x.a < 0 || x.a >= n || x.opa < 0 || x.opa >= (int)H.ops.size() ||
        H.opdim[x.opa] != H.phys[x.a]) {
      err = "tree: bad term (node_a / op_a)";
      return TTNS_EINVAL;
    }
    if (x.b != -1 && (x.b < 0 || x.b >= n || x.b == x.a || x.opb < 0 ||
                      x.opb >= (int)H.ops.size() || H.opdim[x.opb] != H.phys[x.b])) {
      err = "tree: bad term (node_b / op_b)";
      return TTNS_EINVAL;
    }
    if (!std::isfinite(x.coef)) {
      err = "tree: non-finite coefficient";
      return TTNS_ENUMERIC;
    }
  }
  for (size_t k = 0; k < H.obs_node.size(); ++k)
    if (H.obs_node[k] < 0 || H.obs_node[k] >= n || H.obs_op[k] < 0 ||
        H.obs_op[k] >= (int)H.ops.size() || H.opdim[H.obs_op[k]] != H.phys[H.obs_node[k]]) {
      err = "tree: bad observable";
      return TTNS_EINVAL;
    }
  for (int v = 0; v < n; ++v)
    for (const cd& a : H.init[v])
      if (!std::isfinite(a.x) || !std::isfinite(a.y)) {
        err = "tree: non-finite initial state";
        return TTNS_ENUMERIC;
      }
  for (const auto& m : H.ops)
    for (const cd& a : m)
      if (!std::isfinite(a.x) || !std::isfinite(a.y)) {
        err = "tree: non-finite operator";
        return TTNS_ENUMERIC;
      }
  // Hermiticity of the operator sum, per node pair
  {
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (size_t k = 0; k < H.terms.size(); ++k) {
      const HostTerm& x = H.terms[k];
      if (x.b == -1) groups[{x.a, -1}].push_back((int)k);
      else if (x.a < x.b) groups[{x.a, x.b}].push_back((int)k);
    }
    // terms listed with node_a > node_b: swap their ends into the same group
    for (size_t k = 0; k < H.terms.size(); ++k) {
      HostTerm x = H.terms[k];
      if (x.b != -1 && x.a > x.b) {
        H.terms[k] = HostTerm{x.b, x.opb, x.a, x.opa, x.coef};
        groups[{x.b, x.a}].push_back((int)k);
      }
    }
    double scale = 0.0;
    for (const HostTerm& x : H.terms) scale = std::max(scale, std::fabs(x.coef));
    for (auto& g : groups) {
      const double def = herm_defect(t, g.second, g.first.second == -1);
      if (def > 1e-20 * std::max(1.0, scale * scale) * 1e4) {
        err = "tree: the operator sum is not Hermitian (nodes " + std::to_string(g.first.first) +
              ", " + std::to_string(g.first.second) + ")";
        return TTNS_EINVAL;
      }
    }
  }
  // bond dimensions: clamp to what either side can carry (fixed point)
  t.D.assign(n, 0);
  for (int v = 1; v < n; ++v) {
    if (H.bondreq[v] < 1) {
      err = "tree: bond_dim must be >= 1";
      return TTNS_EINVAL;
    }
    t.D[v] = H.bondreq[v];
  }
  for (bool changed = true; changed;) {
    changed = false;
    for (int v = n - 1; v > 0; --v) {
      long long cap = H.phys[v];
      for (int c : t.children[v]) cap = std::min<long long>(cap * t.D[c], 1LL << 40);
      if (t.D[v] > cap) {
        t.D[v] = (int)cap;
        changed = true;
      }
    }
    for (int v = 1; v < n; ++v) {
      const int p = H.parent[v];
      long long cap = (long long)H.phys[p] * (p != 0 ? t.D[p] : 1);
      for (int s : t.children[p])
        if (s != v) cap = std::min<long long>(cap * t.D[s], 1LL << 40);
      if (t.D[v] > cap) {
        t.D[v] = (int)cap;
        changed = true;
      }
    }
  }
  // shapes
  t.shape.assign(n, Shape{});
  t.maxsize = 1;
  t.maxD = 1;
  t.max_rows = 1;
  for (int v = 0; v < n; ++v) {
    std::vector<int> dims;
    if (v) dims.push_back(t.D[v]);
    dims.push_back(H.phys[v]);
    for (int c : t.children[v]) dims.push_back(t.D[c]);
    if ((int)dims.size() > kMaxRank) {
      err = "tree: a node has more than " + std::to_string(kMaxRank - 2) + " children";
      return TTNS_EINVAL;
    }
    Shape& s = t.shape[v];
    s.rank = (int)dims.size();
    s.phys_axis = v == 0 ? 0 : 1;
    long long size = 1;
    for (int a = s.rank - 1; a >= 0; --a) {
      s.dims[a] = dims[a];
      s.stride[a] = (int)size;
      size *= dims[a];
      if (size > (1LL << 30)) {
        err = "tree: node tensor too large";
        return TTNS_EINVAL;
      }
    }
    for (int a = s.rank; a < kMaxRank; ++a) s.dims[a] = 1, s.stride[a] = 1;
    s.size = (int)size;
    t.maxsize = std::max(t.maxsize, s.size);
    for (int a = 0; a < s.rank; ++a) {
      if (a == s.phys_axis) continue;
      if (dims[a] > kMaxD) {
        err = "tree: bond dimension above " + std::to_string(kMaxD);
        return TTNS_EINVAL;
      }
      t.maxD = std::max(t.maxD, dims[a]);
      t.max_rows = std::max(t.max_rows, s.size / dims[a]);
    }
  }
  // operator bands and on-site sums
  t.op_lo.resize(H.ops.size());
  t.op_hi.resize(H.ops.size());
  for (size_t k = 0; k < H.ops.size(); ++k) band_of(H.ops[k], H.opdim[k], t.op_lo[k], t.op_hi[k]);
  t.site.assign(n, {});
  t.site_lo.assign(n, 0);
  t.site_hi.assign(n, 0);
  for (const HostTerm& x : H.terms) {
    if (x.b != -1) continue;
    const int d = H.phys[x.a];
    if (t.site[x.a].empty()) t.site[x.a].assign((size_t)d * d, cd{0, 0});
    for (int i = 0; i < d * d; ++i) {
      t.site[x.a][i].x += x.coef * H.ops[x.opa][i].x;
      t.site[x.a][i].y += x.coef * H.ops[x.opa][i].y;
    }
  }
  for (int v = 0; v < n; ++v)
    if (!t.site[v].empty()) band_of(t.site[v], H.phys[v], t.site_lo[v], t.site_hi[v]);
  // environment channels of every directed edge
  t.env.clear();
  for (int v = 1; v < n; ++v) {
    const int p = H.parent[v];
    for (int dir = 0; dir < 2; ++dir) {
      const int u = dir == 0 ? v : p, w = dir == 0 ? p : v;
      Env e;
      e.D = t.D[v];
      e.keys.push_back(ChanKey{0, 0, 0});
      for (size_t k = 0; k < H.terms.size(); ++k) {
        const HostTerm& x = H.terms[k];
        if (x.b == -1) continue;
        const bool ia = in_side(t, x.a, u, w), ib = in_side(t, x.b, u, w);
        if (ia && !ib) e.keys.push_back(ChanKey{1, (int)k, 0});
        if (ib && !ia) e.keys.push_back(ChanKey{1, (int)k, 1});
      }
      if (dir == 0)  // towards the root: observables below travel up
        for (size_t k = 0; k < H.obs_node.size(); ++k)
          if (in_subtree(t, H.obs_node[k], v)) e.keys.push_back(ChanKey{2, (int)k, 0});
      t.env[{u, w}] = e;
    }
  }
  // temporaries for bond-bond terms and crossing terms per bond
  t.ntmp = 0;
  for (int v = 0; v < n; ++v) {
    int cnt = 0, entries = (int)nbrs(t, v).size();
    for (const HostTerm& x : H.terms) {
      if (x.b == -1) continue;
      const int ra = region(t, v, x.a), rb = region(t, v, x.b);
      if (ra == rb) continue;
      ++entries;
      if (ra != PHYS && rb != PHYS) ++cnt;
    }
    if (entries > kMaxEntries) {
      err = "tree: too many coupling channels at node " + std::to_string(v);
      return TTNS_EINVAL;
    }
    if (cnt > kMaxTmp) {
      err = "tree: too many pass-through terms at node " + std::to_string(v);
      return TTNS_EINVAL;
    }
    t.ntmp = std::max(t.ntmp, cnt);
  }
  for (int v = 1; v < n; ++v) {
    int cnt = 0;
    const Env& e = t.env[{v, H.parent[v]}];
    for (const ChanKey& k : e.keys)
      if (k.kind == 1) ++cnt;
    if (cnt > kMaxPairs) {
      err = "tree: too many terms across the bond above node " + std::to_string(v);
      return TTNS_EINVAL;
    }
  }
  t.kmax = o.krylov_dim;
  t.n_el = H.phys[0];
  t.maxC = std::max(t.maxD, t.n_el);
  t.rec_size = 2 * t.n_el * t.n_el + 2 + (int)H.obs_node.size();
  t.max_nvb = std::max({(t.maxsize + kBlock - 1) / kBlock, kMaxContractVb, kSplitLanes / kBlock});
  return TTNS_OK;
}

// ------------------------------------------------------------------ layout
size_t layout_tree(TreeState& t, size_t off, int rec_cap) {
  auto take = [&](size_t bytes) {
    size_t o = align256(off);
    off = o + std::max<size_t>(bytes, 1);
    return o;
  };
  const size_t C = sizeof(cd);
  const size_t ldv = align256((size_t)t.maxsize * C) / C;
  const size_t D2 = (size_t)t.maxD * t.maxD;
  t.o_scal = take(sizeof(LzScal));
  t.o_counter = take(sizeof(unsigned));
  t.o_rec = take(sizeof(int));
  t.o_stats = take(8 * sizeof(int));
  t.o_V = take((size_t)(t.kmax + 1) * ldv * C);
  t.o_W = take(ldv * C);
  t.o_Z = take(ldv * C);
  t.o_X = take(ldv * C);
  t.o_tmp = take((size_t)std::max(t.ntmp, 1) * ldv * C);
  t.o_R = take(D2 * C);
  t.o_bondV = take((size_t)(t.kmax + 1) * D2 * C);
  t.o_bondW = take(2 * D2 * C);
  t.o_qrA = take(ldv * C);
  t.o_qrQ = take(ldv * C);
  t.o_qrv = take(2 * (size_t)t.max_rows * C);
  t.o_part = take(2 * (size_t)t.max_nvb * kRedStride * C);  // Lanczos buffers A and B
  t.o_cpart = take((size_t)kMaxContractVb * t.maxC * t.maxC * C);
  t.o_qrpart = take((size_t)kMaxQrVb * kQrStride * C);
  t.o_qrs = take(sizeof(QrScal));
  t.o_hist = take((size_t)rec_cap * t.rec_size * sizeof(double));
  t.o_T.resize(t.n);
  for (int v = 0; v < t.n; ++v) t.o_T[v] = take((size_t)t.shape[v].size * C);
  for (auto& kv : t.env) kv.second.off = take(kv.second.keys.size() * (size_t)kv.second.D * kv.second.D * C);
  t.o_opdata.resize(t.ht.ops.size());
  for (size_t k = 0; k < t.ht.ops.size(); ++k) t.o_opdata[k] = take(t.ht.ops[k].size() * C);
  t.o_sitedata.assign(t.n, 0);
  for (int v = 0; v < t.n; ++v)
    if (!t.site[v].empty()) t.o_sitedata[v] = take(t.site[v].size() * C);
  return off;
}

size_t layout_ctx(ttns_ctx& c) {
  size_t off = 0;
  for (auto& t : c.trees) off = layout_tree(t, off, c.opts.record_capacity);
  return off;
}

// ------------------------------------------------------------------ programs
struct Builder {
  ttns_ctx& c;
  TreeState& t;
  int ti;
  std::vector<Op>& out;

  Op base(int type, int nvb) {
    Op o{};
    o.type = type;
    o.nvb = std::max(nvb, 1);
    o.tree = ti;
    o.desc = -1;
    return o;
  }
  static int nvb_of(int n) { return (n + kBlock - 1) / kBlock; }
  // log2 of the lanes per element of a scalar apply over n elements: up to
  // 8, as long as the grid stays within kSplitLanes lanes.  Only the wide
  // executor gains: the one-workgroup executor already has more elements
  // than lanes and would only repeat the dot reductions.
  int apply_lg(int n) const {
    if (c.persistent) return 0;
    int lg = 0;
    while (lg < 3 && ((size_t)n << (lg + 1)) <= (size_t)kSplitLanes) ++lg;
    return lg;
  }
  static int apply_nvb(int n, int lg) { return (int)((((size_t)n << lg) + kBlock - 1) / kBlock); }
  // W = H V_j and its dots (mfma: W already produced by the matrix cores)
  Op lz_op(int v, int j, bool mfma) {
    const int n = t.shape[v].size;
    const int lg = mfma ? 0 : apply_lg(n);
    Op o = base(OP_APPLY_LZ, apply_nvb(n, lg));
    o.desc = t.heff_desc[v];
    o.j = j;
    o.n = n;
    o.i0 = mfma ? 1 : 0;
    o.i1 = lg;
    o.p1 = part_a();
    return o;
  }
  // the two partial-dot buffers of the Lanczos ops (max_nvb slots each)
  cd* part_a() const { return t.dev.partials; }
  cd* part_b() const { return t.dev.partials + (size_t)t.max_nvb * kRedStride; }

  int add_desc(const ApplyDesc& d) {
    c.descs.push_back(d);
    return (int)c.descs.size() - 1;
  }

  ApplyDesc empty_desc(int v, const cd* x, cd* y) {
    ApplyDesc d{};
    d.sh = t.shape[v];
    d.x = x;
    d.y = y;
    d.site = nullptr;
    d.site_coef = 1.0;
    d.n_entries = 0;
    return d;
  }

  void count_flops(ApplyDesc& d) {
    // complex multiply-adds of the operator-sum form: every row s of a
    // banded physical operator contributes its nonzeros; bond products D each
    const Shape& sh = d.sh;
    const int dp = sh.dims[sh.phys_axis];
    const double per_s = (double)sh.size / dp;
    auto row_nnz = [&](const cd* op, int lo, int hi, int s) {
      if (!op) return 1.0;
      return (double)(std::min(hi, dp - 1 - s) - std::max(lo, -s) + 1);
    };
    double macs = 0.0;
    for (int s = 0; s < dp; ++s) {
      if (d.site) macs += per_s * row_nnz(d.site, d.site_lo, d.site_hi, s);
      for (int k = 0; k < d.n_entries; ++k)
        macs += per_s * row_nnz(d.e[k].op, d.e[k].op_lo, d.e[k].op_hi, s) * sh.dims[d.e[k].axis];
    }
    d.flops = 8.0 * macs;
  }

  void add_entry(ApplyDesc& d, int axis, const cd* E, const cd* op, int lo, int hi, double coef, int src) {
    Entry& e = d.e[d.n_entries++];
    e.axis = axis;
    e.src = src;
    e.E = E;
    e.op = op;
    e.op_lo = lo;
    e.op_hi = hi;
    e.coef = coef;
  }

  // Sum of the terms of H acting inside v's regions except `exclude`
  // (exclude = -2: the full H_eff at v).  Bond-bond terms need a first mode
  // product into a temporary: returned as pre-stage descriptors.
  ApplyDesc make_sum(int v, int exclude, const cd* x, cd* y, std::vector<ApplyDesc>& pre) {
    ApplyDesc d = empty_desc(v, x, y);
    if (!t.site[v].empty()) {
      d.site = t.sitedev[v];
      d.site_lo = t.site_lo[v];
      d.site_hi = t.site_hi[v];
    }
    for (int w : nbrs(t, v)) {
      if (w == exclude) continue;
      add_entry(d, axis_of(t, v, w), t.env[{w, v}].chan(ChanKey{0, 0, 0}), nullptr, 0, 0, 1.0, -1);
    }
    int ntmp = 0;
    const auto& H = t.ht;
    for (size_t k = 0; k < H.terms.size(); ++k) {
      const HostTerm& x_ = H.terms[k];
      if (x_.b == -1) continue;
      const int ra = region(t, v, x_.a), rb = region(t, v, x_.b);
      if (ra == rb || ra == exclude || rb == exclude) continue;
      if (ra == PHYS) {
        add_entry(d, axis_of(t, v, rb), t.env[{rb, v}].chan(ChanKey{1, (int)k, 1}), t.opdev[x_.opa],
                  t.op_lo[x_.opa], t.op_hi[x_.opa], x_.coef, -1);
      } else if (rb == PHYS) {
        add_entry(d, axis_of(t, v, ra), t.env[{ra, v}].chan(ChanKey{1, (int)k, 0}), t.opdev[x_.opb],
                  t.op_lo[x_.opb], t.op_hi[x_.opb], x_.coef, -1);
      } else {
        ApplyDesc p = empty_desc(v, x, t.dev.tmp[ntmp]);
        add_entry(p, axis_of(t, v, rb), t.env[{rb, v}].chan(ChanKey{1, (int)k, 1}), nullptr, 0, 0,
                  1.0, -1);
        count_flops(p);
        pre.push_back(p);
        d.tmp[ntmp] = t.dev.tmp[ntmp];
        add_entry(d, axis_of(t, v, ra), t.env[{ra, v}].chan(ChanKey{1, (int)k, 0}), nullptr, 0, 0,
                  x_.coef, ntmp);
        ++ntmp;
      }
    }
    count_flops(d);
    return d;
  }

  int sum_desc(int v, int exclude, const cd* x, cd* y, std::vector<int>& pre) {
    std::vector<ApplyDesc> pd;
    ApplyDesc d = make_sum(v, exclude, x, y, pd);
    for (auto& p : pd) pre.push_back(add_desc(p));
    return add_desc(d);
  }

  // H_eff at v as matrix-core groups; false when v does not qualify.
  // node class of the autotuner: shape, physical axis and term structure
  std::string heff_key(int v, const ApplyDesc& d, size_t n_pre) const {
    const Shape& sh = t.shape[v];
    std::string k = "node";
    for (int a = 0; a < sh.rank; ++a) k += (a ? "x" : " ") + std::to_string(sh.dims[a]);
    k += " phys" + std::to_string(sh.phys_axis) + " terms" + std::to_string(d.n_entries) + "/" +
         std::to_string(n_pre);
    return k;
  }

  bool plan_mode_groups(int v) {
    const int prec = c.opts.precision;
    const Shape& sh = t.shape[v];
    // the one-workgroup executor runs the reduced-precision forms on the
    // matrix cores with the small operand tile and 16-column blocks (bonds
    // up to 32) and keeps the scalar FP64 apply otherwise
    if (c.persistent && prec == TTNS_FP64) return false;
    const int maxD = c.persistent ? 32 : mode_max_bond(prec);
    for (int a = 0; a < sh.rank; ++a)
      if (a != sh.phys_axis && sh.dims[a] > maxD) return false;
    std::vector<ApplyDesc> pre;
    ApplyDesc d = make_sum(v, -2, t.T[v], t.dev.W, pre);
    if (d.n_entries == 0) return false;
    t.mode_tile[v] = 0;
    if (c.persistent) {
      t.mode_tile[v] = 1 | 4;  // small operands, 16 columns
    } else if (!c.tune_probe) {
      auto it = c.tune_heff.find(heff_key(v, d, pre.size()));
      if (it != c.tune_heff.end()) {
        if (it->second == 0) return false;
        t.mode_tile[v] = it->second;
      } else if (sh.size < kMfmaMinSize && !(c.opts.flags & TTNS_FLAG_MFMA_ALL)) {
        return false;  // small nodes: latency-bound, scalar FP64 apply
      }
    }
    auto blank = [&](const cd* src, cd* y) {
      ModeDesc m{};
      m.sh = sh;
      m.prec = prec;
      m.src = src;
      m.x = t.T[v];
      m.y = y;
      m.site_coef = 1.0;
      m.n_rest = sh.size / sh.dims[sh.phys_axis];
      return m;
    };
    auto add_term = [&](ModeDesc& m, const Entry& e) -> bool {
      if (m.n_e >= kMaxGroup) return false;
      const int k = m.n_e++;
      m.E[k] = e.E;
      m.op[k] = e.op;
      m.lo[k] = e.op ? e.op_lo : 0;
      m.hi[k] = e.op ? e.op_hi : 0;
      m.coef[k] = e.coef;
      m.band_lo = k == 0 ? m.lo[k] : std::min(m.band_lo, m.lo[k]);
      m.band_hi = k == 0 ? m.hi[k] : std::max(m.band_hi, m.hi[k]);
      return true;
    };
    // host copy of a term's local operator (null: identity)
    auto host_op = [&](const cd* dev) -> const std::vector<cd>* {
      for (size_t k = 0; k < t.opdev.size(); ++k)
        if (t.opdev[k] == dev) return &t.ht.ops[k];
      return nullptr;
    };
    // algorithmic flops: one complex D x D by D x n_rest product per term and
    // output physical index s whose band holds a nonzero weight (what the
    // kernel multiplies on the matrix cores)
    auto finish = [&](ModeDesc& m) {
      m.n_rest = sh.size / (sh.dims[m.axis] * sh.dims[sh.phys_axis]);
      const double D = sh.dims[m.axis];
      const int dp = sh.dims[sh.phys_axis];
      int active = 0;
      for (int e = 0; e < m.n_e; ++e) {
        const std::vector<cd>* op = m.op[e] ? host_op(m.op[e]) : nullptr;
        for (int s = 0; s < dp; ++s) {
          if (!m.op[e]) {
            ++active;
            continue;
          }
          bool any = false;
          for (int o = std::max(m.lo[e], -s); o <= std::min(m.hi[e], dp - 1 - s); ++o) {
            const cd g = op ? (*op)[(size_t)s * dp + s + o] : cd{1, 0};
            any = any || g.x != 0.0 || g.y != 0.0;
          }
          active += any;
        }
      }
      m.flops = 8.0 * D * D * m.n_rest * active;
    };
    std::vector<ModeDesc> groups;
    std::vector<int> gkey_axis, gkey_src;
    for (int k = 0; k < d.n_entries; ++k) {
      const Entry& e = d.e[k];
      int g = -1;
      for (size_t i = 0; i < groups.size(); ++i)
        if (gkey_axis[i] == e.axis && gkey_src[i] == e.src) g = (int)i;
      if (g < 0) {
        groups.push_back(blank(e.src < 0 ? t.T[v] : t.dev.tmp[e.src], t.dev.W));
        groups.back().axis = e.axis;
        gkey_axis.push_back(e.axis);
        gkey_src.push_back(e.src);
        g = (int)groups.size() - 1;
      }
      if (!add_term(groups[g], e)) return false;
    }
    // the first group writes W and carries the on-site term: it must read x
    int first = -1;
    for (size_t i = 0; i < groups.size(); ++i)
      if (gkey_src[i] < 0) {
        first = (int)i;
        break;
      }
    if (first < 0) return false;
    std::swap(groups[0], groups[first]);
    std::swap(gkey_src[0], gkey_src[first]);
    groups[0].site = d.site;
    groups[0].site_lo = d.site_lo;
    groups[0].site_hi = d.site_hi;
    groups[0].site_coef = d.site_coef;
    for (size_t i = 1; i < groups.size(); ++i) groups[i].accumulate = 1;
    std::vector<int> pre_ids, grp_ids;
    for (size_t i = 0; i < pre.size(); ++i) {
      // pre-stage: a single mode product into tmp[i]
      ModeDesc m = blank(t.T[v], t.dev.tmp[i]);
      m.axis = pre[i].e[0].axis;
      if (!add_term(m, pre[i].e[0])) return false;
      finish(m);
      c.modes.push_back(m);
      pre_ids.push_back((int)c.modes.size() - 1);
    }
    for (size_t i = 0; i < groups.size(); ++i) {
      finish(groups[i]);
      if (gkey_src[i] >= 0) groups[i].src = t.dev.tmp[gkey_src[i]];
      c.modes.push_back(groups[i]);
      grp_ids.push_back((int)c.modes.size() - 1);
    }
    t.mode_pre[v] = pre_ids;
    t.mode_groups[v] = grp_ids;
    return true;
  }

  // launches of one matrix-core H_eff apply: input x (V_j or a caller
  // buffer), output y (W or a caller buffer)
  void mode_apply(int v, const cd* x, cd* y) {
    for (int id : t.mode_pre[v]) {
      const ModeDesc& m = c.modes[id];
      Op o = base(OP_MODE, 1);
      o.desc = id;
      o.p0 = x;
      o.p1 = nullptr;
      o.i0 = m.prec;
      o.n = m.n_rest;
      o.axis = m.sh.dims[m.sh.phys_axis];
      o.j = mode_padded(m.prec, m.sh.dims[m.axis]);
      o.i1 = t.mode_tile[v];
      out.push_back(o);
    }
    for (int id : t.mode_groups[v]) {
      const ModeDesc& m = c.modes[id];
      Op o = base(OP_MODE, 1);
      o.desc = id;
      const bool from_x = m.src == t.T[v];
      o.p0 = from_x ? x : nullptr;
      o.p1 = y;
      o.i0 = m.prec;
      o.n = m.n_rest;
      o.axis = m.sh.dims[m.sh.phys_axis];
      o.j = mode_padded(m.prec, m.sh.dims[m.axis]);
      o.i1 = t.mode_tile[v];
      out.push_back(o);
    }
  }

  // The factor of channel `key` of E_{u->w} acting on u's tensor.
  int chan_desc(int u, const ChanKey& key, const cd* x, cd* y) {
    ApplyDesc d = empty_desc(u, x, y);
    const auto& H = t.ht;
    int node, op;
    if (key.kind == 1) {
      const HostTerm& x_ = H.terms[key.k];
      node = key.end == 0 ? x_.a : x_.b;
      op = key.end == 0 ? x_.opa : x_.opb;
    } else {
      node = H.obs_node[key.k];
      op = H.obs_op[key.k];
    }
    const int r = region(t, u, node);
    if (r == PHYS) {
      d.site = t.opdev[op];
      d.site_lo = t.op_lo[op];
      d.site_hi = t.op_hi[op];
    } else {
      add_entry(d, axis_of(t, u, r), t.env[{r, u}].chan(key), nullptr, 0, 0, 1.0, -1);
    }
    count_flops(d);
    return add_desc(d);
  }

  int make_bond_desc(int u, int w) {
    BondDesc b{};
    const Env& eu = t.env[{u, w}];
    const Env& ev = t.env[{w, u}];
    b.Du = eu.D;
    b.Dv = ev.D;
    b.R = t.dev.R;
    b.Eu = eu.chan(ChanKey{0, 0, 0});
    b.Ev = ev.chan(ChanKey{0, 0, 0});
    const auto& H = t.ht;
    for (size_t k = 0; k < H.terms.size(); ++k) {
      const HostTerm& x_ = H.terms[k];
      if (x_.b == -1) continue;
      const bool ia = in_side(t, x_.a, u, w), ib = in_side(t, x_.b, u, w);
      if (ia == ib) continue;
      const int eu_end = ia ? 0 : 1;
      b.coef[b.n_pairs] = x_.coef;
      b.Euk[b.n_pairs] = eu.chan(ChanKey{1, (int)k, eu_end});
      b.Evk[b.n_pairs] = ev.chan(ChanKey{1, (int)k, 1 - eu_end});
      ++b.n_pairs;
    }
    c.bonds.push_back(b);
    return (int)c.bonds.size() - 1;
  }

  // Every descriptor the programs of this tree use, created once.
  void plan_all() {
    t.heff_desc.assign(t.n, -1);
    t.heff_pre.assign(t.n, {});
    t.mode_pre.assign(t.n, {});
    t.mode_groups.assign(t.n, {});
    t.mode_tile.assign(t.n, 0);
    for (int v = 0; v < t.n; ++v) {
      t.heff_desc[v] = sum_desc(v, -2, t.T[v], t.dev.W, t.heff_pre[v]);
      plan_mode_groups(v);
    }
    for (auto& kv : t.env) {
      const int u = kv.first.first, w = kv.first.second;
      TreeState::EdgePlan& ep = t.edge[{u, w}];
      for (const ChanKey& key : kv.second.keys) {
        if (key.kind == 0) ep.chan_desc.push_back(sum_desc(u, w, t.T[u], t.dev.Z, ep.h_pre));
        else ep.chan_desc.push_back(chan_desc(u, key, t.T[u], t.dev.Z));
      }
      ApplyDesc d = empty_desc(w, t.T[w], t.dev.X);
      add_entry(d, axis_of(t, w, u), t.dev.R, nullptr, 0, 0, 1.0, -1);
      count_flops(d);
      ep.absorb_desc = add_desc(d);
      ep.bond_desc = make_bond_desc(u, w);
    }
    t.obs_desc.clear();
    for (size_t k = 0; k < t.ht.obs_node.size(); ++k) {
      const int node = t.ht.obs_node[k];
      ApplyDesc d = empty_desc(0, t.T[0], t.dev.Z);
      const int r = region(t, 0, node);
      if (r == PHYS) {
        d.site = t.opdev[t.ht.obs_op[k]];
        d.site_lo = t.op_lo[t.ht.obs_op[k]];
        d.site_hi = t.op_hi[t.ht.obs_op[k]];
      } else {
        add_entry(d, axis_of(t, 0, r), t.env[{r, 0}].chan(ChanKey{2, (int)k, 0}), nullptr, 0, 0,
                  1.0, -1);
      }
      count_flops(d);
      t.obs_desc.push_back(add_desc(d));
    }
  }

  void apply_op(int desc, const cd* x_override = nullptr) {
    const int n = c.descs[desc].sh.size;
    const int lg = apply_lg(n);
    Op o = base(OP_APPLY, apply_nvb(n, lg));
    o.desc = desc;
    o.i1 = lg;
    o.p0 = x_override;
    out.push_back(o);
  }

  // E_{u->w} for every channel, with u's tensor already an isometry towards w.
  void env_update(int u, int w) {
    Env& e = t.env[{u, w}];
    const TreeState::EdgePlan& ep = t.edge[{u, w}];
    const int ax = axis_of(t, u, w);
    const Shape& sh = t.shape[u];
    const int rows = sh.size / sh.dims[ax];
    const int nvb = std::min(kMaxContractVb, std::max(1, (rows + 31) / 32));
    for (size_t i = 0; i < e.keys.size(); ++i) {
      if (e.keys[i].kind == 0)
        for (int p : ep.h_pre) apply_op(p);
      apply_op(ep.chan_desc[i]);
      Op o = base(OP_CONTRACT, nvb);
      o.desc = ep.chan_desc[i];
      o.axis = ax;
      o.p0 = t.T[u];
      o.p2 = t.dev.Z;
      o.p1 = e.base + i * (size_t)e.D * e.D;
      o.i0 = 0;
      out.push_back(o);
    }
  }

  // Guarded QR of u's tensor towards neighbour w (or its parent axis when
  // w = -1): one workgroup with the matrix in LDS when it fits, else the
  // phased multi-workgroup form.
  void qr_axis(int u, int ax) {
    const Shape& sh = t.shape[u];
    const int cols = sh.dims[ax], rows = sh.size / cols;
    Op o = base(OP_QR, 1);
    o.desc = t.heff_desc[u];  // shape
    o.axis = ax;
    o.p1 = t.T[u];
    // one workgroup (LDS-resident, or streaming through L2 up to
    // kQrOneGroupRows rows); taller matrices split rows over workgroups with
    // one launch per phase and column
    const bool lds = (size_t)rows * (cols + 2) <= (size_t)kQrLdsEntries;
    int choice = -1;  // -1: default rule
    if (!lds && !c.tune_probe) {
      auto it = c.tune_qr.find(qr_key(rows, cols));
      if (it != c.tune_qr.end()) choice = it->second;
    }
    if (lds || choice == 0 || (choice < 0 && rows <= kQrOneGroupRows)) {
      // the 512-thread kernel with Q in LDS when it fits (the one-workgroup
      // executor keeps the op's own workgroup)
      o.i1 = (!c.persistent && qr_fast_fits(rows, cols)) ? 1 : 0;
      out.push_back(o);
      return;
    }
    push_wide_qr(out, o, cols, choice > 0 ? choice : qr_wide_default(rows));
  }
  // the launches of a wide QR with nvb workgroups (o: the OP_QR op)
  static void push_wide_qr(std::vector<Op>& out, Op o, int cols, int nvb) {
    o.type = OP_QRW;
    o.nvb = nvb;
    o.i0 = 0;
    out.push_back(o);
    for (int k = 0; k < cols; ++k)
      for (int ph = 1; ph <= 5; ++ph) {
        o.i0 = ph;
        o.j = k;
        out.push_back(o);
      }
    o.i0 = 6;
    o.j = cols - 1;
    out.push_back(o);
  }
  void qr(int u, int w) { qr_axis(u, axis_of(t, u, w)); }
  static std::string qr_key(int rows, int cols) {
    return "qr " + std::to_string(rows) + "x" + std::to_string(cols);
  }
  static int qr_wide_default(int rows) { return std::min(kMaxQrVb, std::max(1, (rows + 511) / 512)); }

  // x (node v's tensor or the absorb buffer) -> T[v] = exp(-i h H_eff) x
  void evolve_node(int v, const cd* x) {
    const int n = t.shape[v].size;
    Op o = base(OP_NORM, nvb_of(n));
    o.p0 = x;
    o.n = n;
    out.push_back(o);
    o = base(OP_SCALE, nvb_of(n));
    o.p0 = x;
    o.n = n;
    out.push_back(o);
    const int kk = std::min(t.kmax, n);
    const bool mfma = !t.mode_groups[v].empty();
    for (int j = 0; j < kk; ++j) {
      const cd* vj = t.dev.V + (size_t)j * t.dev.ldv;
      if (mfma) {
        mode_apply(v, vj, t.dev.W);
      } else {
        for (int p : t.heff_pre[v]) apply_op(p, vj);
      }
      // partial dots: OP_APPLY_LZ -> buffer A -> OP_ORTH1 -> buffer B ->
      // OP_ORTH2, each consumer folding its producer's partials
      const Op a = lz_op(v, j, mfma);
      out.push_back(a);
      o = base(OP_ORTH1, nvb_of(n));
      o.j = j;
      o.n = n;
      o.p2 = part_a();
      o.i0 = a.nvb;
      o.p1 = part_b();
      out.push_back(o);
      const int nvb1 = o.nvb;
      o = base(OP_ORTH2, nvb_of(n));
      o.j = j;
      o.n = n;
      o.p2 = part_b();
      o.i0 = nvb1;
      out.push_back(o);
    }
    o = base(OP_COMBINE, nvb_of(n));
    o.sign = -1;
    o.n = n;
    o.p1 = t.T[v];
    out.push_back(o);
  }

  // centre u -> neighbour w: QR, environment, optional backward bond step,
  // absorb R into w.  With evolve_next the absorbed tensor is left in X for
  // the following node evolution; otherwise it is copied into w's tensor.
  void move(int u, int w, bool bond_step, bool leave_in_x = false) {
    const TreeState::EdgePlan& ep = t.edge[{u, w}];
    qr(u, w);
    env_update(u, w);
    if (bond_step) {
      Op o = base(OP_BOND, 1);
      o.desc = ep.bond_desc;
      o.sign = +1;
      o.i0 = t.maxD * t.maxD;
      // the 512-thread kernel with everything in LDS when it fits (the
      // one-workgroup executor keeps the op's own workgroup)
      const BondDesc& bd = c.bonds[ep.bond_desc];
      o.i1 = (!c.persistent && bond_fast_fits(bd.Du, bd.Dv, c.opts.krylov_dim, bd.n_pairs)) ? 1 : 0;
      out.push_back(o);
    }
    apply_op(ep.absorb_desc);
    if (!leave_in_x) {
      Op o = base(OP_COPY, nvb_of(t.shape[w].size));
      o.p0 = t.dev.X;
      o.p1 = t.T[w];
      o.n = t.shape[w].size;
      out.push_back(o);
    }
    t.centre = w;
  }

  std::vector<int> path(int a, int b) {
    std::vector<int> ua{a}, ub{b};
    while (ua.back() != 0) ua.push_back(parent_of(t, ua.back()));
    while (ub.back() != 0) ub.push_back(parent_of(t, ub.back()));
    int lca = 0;
    for (int x : ua)
      if (std::find(ub.begin(), ub.end(), x) != ub.end()) {
        lca = x;
        break;
      }
    std::vector<int> p;
    for (int x : ua) {
      p.push_back(x);
      if (x == lca) break;
    }
    std::vector<int> tail;
    for (int x : ub) {
      if (x == lca) break;
      tail.push_back(x);
    }
    p.insert(p.end(), tail.rbegin(), tail.rend());
    return p;
  }

  void move_to(int target) {
    std::vector<int> p = path(t.centre, target);
    for (size_t i = 0; i + 1 < p.size(); ++i) move(p[i], p[i + 1], false);
  }

  // pre-order sweep: node first, then every child (the centre returns to v
  // between children)
  void pre(int v, bool from_x) {
    evolve_node(v, from_x ? t.dev.X : t.T[v]);
    const auto& ch = t.children[v];
    for (size_t i = 0; i < ch.size(); ++i) {
      move(v, ch[i], true, true);
      pre(ch[i], true);
      if (i + 1 < ch.size()) move_to(v);
    }
  }

  // adjoint post-order sweep
  void post(int v) {
    const auto& ch = t.children[v];
    for (int i = (int)ch.size() - 1; i >= 0; --i) {
      if (i + 1 < (int)ch.size()) move_to(ch[i] + t.sub[ch[i]] - 1);
      post(ch[i]);
      move(ch[i], v, true);
    }
    evolve_node(v, t.T[v]);
  }

  void observe(bool count_step) {
    const int n_el = t.n_el;
    const int root_size = t.shape[0].size;
    {
      Op o = base(OP_CONTRACT, std::min(kMaxContractVb, std::max(1, (root_size / n_el + 31) / 32)));
      o.desc = t.heff_desc[0];
      o.axis = 0;
      o.p0 = t.T[0];
      o.p2 = t.T[0];
      o.i0 = 1;
      o.i1 = 0;
      out.push_back(o);
    }
    // energy <C|H_eff C>
    apply_op(t.heff_desc[0], t.T[0]);
    {
      Op o = base(OP_DOT, nvb_of(root_size));
      o.p0 = t.T[0];
      o.p2 = c.descs[t.heff_desc[0]].y;
      o.n = root_size;
      o.i1 = 2 * n_el * n_el + 1;
      out.push_back(o);
    }
    // recorded local observables: <C| E_obs(axis) C> at the root
    for (size_t k = 0; k < t.obs_desc.size(); ++k) {
      apply_op(t.obs_desc[k]);
      Op o = base(OP_DOT, nvb_of(root_size));
      o.p0 = t.T[0];
      o.p2 = t.dev.Z;
      o.n = root_size;
      o.i1 = 2 * n_el * n_el + 2 + (int)k;
      out.push_back(o);
    }
    Op o = base(OP_RECORD, 1);
    o.i0 = n_el;
    o.i1 = 2 * n_el * n_el;
    o.j = count_step ? 1 : 0;
    out.push_back(o);
  }
};

// ------------------------------------------------------------------ execution
// Kernel id, algorithmic flops and bytes of one launch (for profiling).
void op_cost(const ttns_ctx& c, const Op& o, int& kid, double& flops, double& bytes) {
  const double C = 16.0;
  flops = bytes = 0.0;
  kid = o.type == OP_MODE ? TTNS_K_MODE_FP64 + o.i0 : o.type;
  switch (o.type) {
    case OP_APPLY_LZ: {
      const ApplyDesc& d = c.descs[o.desc];
      if (o.i0) {  // only the dots of an MFMA apply
        flops = 8.0 * d.sh.size * (o.j + 2);
        bytes = C * d.sh.size * (o.j + 2);
      } else {
        flops = d.flops + 8.0 * d.sh.size * (o.j + 2);
        bytes = C * d.sh.size * (o.j + 3);
      }
      return;
    }
    case OP_MODE: {
      const ModeDesc& m = c.modes[o.desc];
      const double D = m.sh.dims[m.axis];
      flops = m.flops;
      bytes = C * m.sh.size * ((m.band_hi - m.band_lo + 1) + 1 + m.accumulate) + C * D * D * m.n_e;
      return;
    }
    case OP_NORM:
    case OP_SCALE:
    case OP_COMBINE:
    case OP_ORTH1:
    case OP_ORTH2: {
      const double n = o.n, k = o.type == OP_COMBINE ? c.opts.krylov_dim : o.j + 1;
      flops = 8.0 * n * (o.type == OP_ORTH1 ? 2 * k : k);
      bytes = C * n * (k + 1);
      return;
    }
    case OP_QR:
    case OP_QRW: {
      if (o.type == OP_QRW && o.i0 != 0) return;  // counted once per QR
      const Shape& sh = c.descs[o.desc].sh;
      const double cols = sh.dims[o.axis], rows = sh.size / cols;
      flops = 16.0 * rows * cols * cols;
      bytes = 2.0 * C * rows * cols;
      return;
    }
    case OP_CONTRACT: {
      const Shape& sh = c.descs[o.desc].sh;
      const double D = sh.dims[o.axis];
      flops = 8.0 * sh.size * D;
      bytes = 2.0 * C * sh.size + C * D * D;
      return;
    }
    case OP_APPLY: {
      const ApplyDesc& d = c.descs[o.desc];
      flops = d.flops;
      bytes = 2.0 * C * d.sh.size;
      return;
    }
    case OP_BOND: {
      const BondDesc& b = c.bonds[o.desc];
      const double Du = b.Du, Dv = b.Dv;
      flops = 8.0 * c.opts.krylov_dim * (Du * Du * Dv + Du * Dv * Dv) * (1 + b.n_pairs);
      bytes = C * (2.0 * Du * Dv + (Du * Du + Dv * Dv) * (1 + b.n_pairs));
      return;
    }
    case OP_COPY:
      bytes = 2.0 * C * o.n;
      return;
    default:
      return;
  }
}

int run_ops(ttns_ctx& c, const std::vector<Op>& ops) {
  for (const Op& o : ops) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c.profile) {
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      HIPCHK(hipEventRecord(e0, c.stream));
    }
    HIPCHK(launch_op(o, c.tables, c.stream));
    if (c.profile) {
      HIPCHK(hipEventRecord(e1, c.stream));
      ttns_ctx::Pending p{e0, e1, 0, 0.0, 0.0};
      op_cost(c, o, p.cls, p.flops, p.bytes);
      c.ev_pool.push_back(p);
    }
  }
  return TTNS_OK;
}

int drain_profile(ttns_ctx& c) {
  if (c.ev_pool.empty()) return TTNS_OK;
  HIPCHK(hipStreamSynchronize(c.stream));
  for (auto& pr : c.ev_pool) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, pr.e0, pr.e1));
    c.cls_ms[pr.cls] += ms;
    c.cls_flops[pr.cls] += pr.flops;
    c.cls_bytes[pr.cls] += pr.bytes;
    c.cls_n[pr.cls] += 1;
    (void)hipEventDestroy(pr.e0);
    (void)hipEventDestroy(pr.e1);
  }
  c.ev_pool.clear();
  return TTNS_OK;
}

int set_half(ttns_ctx& c, double h) {
  HIPCHK(launch_set_half_step(c.tables.half_step, h, c.stream));
  c.last_h = h;
  return TTNS_OK;
}

// Host -> device copy on the context stream, completed before returning (the
// host buffers are temporaries).
int upload(ttns_ctx& c, size_t off, const void* src, size_t bytes) {
  if (bytes == 0) return TTNS_OK;
  HIPCHK(hipMemcpyAsync(c.ws + off, src, bytes, hipMemcpyHostToDevice, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  return TTNS_OK;
}

constexpr int kScratchDescs = 1 + kMaxTmp;  // ttns_apply_heff: H_eff + pre-stages

int validate_program(ttns_ctx& c, const std::vector<Op>& ops, bool allow_user_xy);
// programs whose inputs and outputs are workspace buffers other than the
// planned ones (the energy-surface projections)
int validate_program_aux(ttns_ctx& c, const std::vector<Op>& ops) { return validate_program(c, ops, true); }

void set_tree_pointers(ttns_ctx& c, TreeState& t, char* base) {
  auto P = [&](size_t o_) { return (cd*)(base + o_); };
  TreeDev& d = t.dev;
  const size_t ldv = align256((size_t)t.maxsize * sizeof(cd)) / sizeof(cd);
  d.scal = (LzScal*)(base + t.o_scal);
  d.counter = (unsigned*)(base + t.o_counter);
  d.rec_count = (int*)(base + t.o_rec);
  d.stats = (int*)(base + t.o_stats);
  d.ldv = (int)ldv;
  d.V = P(t.o_V);
  d.W = P(t.o_W);
  d.Z = P(t.o_Z);
  d.X = P(t.o_X);
  for (int k = 0; k < kMaxTmp; ++k) d.tmp[k] = k < std::max(t.ntmp, 1) ? P(t.o_tmp) + k * ldv : nullptr;
  d.R = P(t.o_R);
  d.bondV = P(t.o_bondV);
  d.bondW = P(t.o_bondW);
  d.qrA = P(t.o_qrA);
  d.qrQ = P(t.o_qrQ);
  d.qrv = P(t.o_qrv);
  d.partials = P(t.o_part);
  d.cpart = P(t.o_cpart);
  d.qrpart = P(t.o_qrpart);
  d.qrs = (QrScal*)(base + t.o_qrs);
  d.hist = (double*)(base + t.o_hist);
  d.max_rows = t.max_rows;
  d.rec_size = t.rec_size;
  d.rec_cap = c.opts.record_capacity;
  d.kmax = c.opts.krylov_dim;
  d.btol = c.opts.breakdown_tol;
  d.rtol = c.opts.rank_tol;
  t.T.resize(t.n);
  for (int v = 0; v < t.n; ++v) t.T[v] = P(t.o_T[v]);
  for (auto& kv : t.env) kv.second.base = P(kv.second.off);
  t.opdev.resize(t.ht.ops.size());
  for (size_t k = 0; k < t.ht.ops.size(); ++k) t.opdev[k] = P(t.o_opdata[k]);
  t.sitedev.assign(t.n, nullptr);
  for (int v = 0; v < t.n; ++v)
    if (!t.site[v].empty()) t.sitedev[v] = P(t.o_sitedata[v]);
}

int prepare(ttns_ctx& c, std::vector<TreeState>&& trees, const ttns_opts* opts, void* ws,
            size_t ws_bytes, void* stream, bool size_only, size_t* bytes_out) {
  ttns_opts o;
  ttns_default_opts(&o);
  if (opts) o = *opts;
  if (o.krylov_dim < 1 || o.krylov_dim > kMaxKrylov) return fail(TTNS_EINVAL, "krylov_dim must be in [1, 16]");
  if (o.record_capacity < 1) return fail(TTNS_EINVAL, "record_capacity must be >= 1");
  if (!(o.rank_tol > 0) || !(o.breakdown_tol > 0)) return fail(TTNS_EINVAL, "tolerances must be > 0");
  if (o.precision < TTNS_FP64 || o.precision > TTNS_BF16X3) return fail(TTNS_EINVAL, "bad precision");
  if (o.executor < TTNS_EXEC_AUTO || o.executor > TTNS_EXEC_PERSISTENT) return fail(TTNS_EINVAL, "bad executor");
  if (o.flags & ~(TTNS_FLAG_MFMA_ALL | TTNS_FLAG_AUTOTUNE)) return fail(TTNS_EINVAL, "unknown option flags");
  c.opts = o;
  c.trees = std::move(trees);
  c.persistent = (o.executor == TTNS_EXEC_PERSISTENT) ||
                 (o.executor == TTNS_EXEC_AUTO && c.trees.size() > 1);
  for (auto& t : c.trees) {
    std::string err;
    int rc = analyze(t, o, err);
    if (rc) return fail(rc, err);
  }
  size_t off = layout_ctx(c);
  // Planning needs the absolute device addresses of the tree data; for a
  // size query any base will do (the descriptors are discarded).
  char* base = size_only ? (char*)(uintptr_t)4096 : (char*)ws;
  if (!size_only) {
    if (!ws) return fail(TTNS_EINVAL, "workspace pointer is null");
    if (((uintptr_t)ws & 255) != 0) return fail(TTNS_EINVAL, "workspace must be 256-byte aligned");
  }
  c.ws = base;
  for (auto& t : c.trees) set_tree_pointers(c, t, base);
  // context-wide half step lives right after the tree data
  off = align256(off);
  c.o_half = off;
  off += 256;
  c.tables.half_step = (double*)(base + c.o_half);
  // energy surfaces / entropy scratch: two matrices of the eigensolver's
  // largest size, its eigenvalues and the partial sums of the projections
  c.o_aux = align256(off);
  off = c.o_aux + aux_bytes();
  // plan: descriptors, init program and one step program per tree
  std::vector<Op> init_ops, persistent_prog;
  c.tree_begin.assign(c.trees.size(), 0);
  c.tree_end.assign(c.trees.size(), 0);
  for (size_t ti = 0; ti < c.trees.size(); ++ti) {
    TreeState& t = c.trees[ti];
    std::vector<Op> ops;
    Builder b{c, t, (int)ti, ops};
    b.plan_all();
    for (int v = t.n - 1; v > 0; --v) b.qr_axis(v, 0);  // isometries towards the parents
    for (int v = t.n - 1; v > 0; --v) b.env_update(v, parent_of(t, v));
    b.observe(false);
    init_ops.insert(init_ops.end(), ops.begin(), ops.end());
    ops.clear();
    t.centre = 0;
    b.pre(0, false);
    b.post(0);
    b.observe(true);
    t.centre = 0;
    c.tree_begin[ti] = (int)persistent_prog.size();
    persistent_prog.insert(persistent_prog.end(), ops.begin(), ops.end());
    c.tree_end[ti] = (int)persistent_prog.size();
  }
  // algorithmic flops of one step per tree (8 real flops per complex
  // multiply-add): H_eff contractions, environment applies and contractions,
  // classical Gram-Schmidt QR (two passes of project + subtract), bond steps
  c.step_flops.assign(c.trees.size(), 0.0);
  c.heff_flops.assign(c.trees.size(), 0.0);
  for (const Op& o : persistent_prog) {
    double f = 0.0, fh = 0.0;
    switch (o.type) {
      case OP_APPLY:
        f = c.descs[o.desc].flops;
        break;
      case OP_APPLY_LZ:
        if (!o.i0) f = fh = c.descs[o.desc].flops;
        break;
      case OP_MODE:
        f = fh = c.modes[o.desc].flops;
        break;
      case OP_CONTRACT: {
        const Shape& sh = c.descs[o.desc].sh;
        const double D = sh.dims[o.axis];
        f = 8.0 * sh.size * D;
        break;
      }
      case OP_QR: {
        const Shape& sh = c.descs[o.desc].sh;
        const double cols = sh.dims[o.axis], rows = sh.size / cols;
        f = 16.0 * rows * cols * cols;
        break;
      }
      case OP_QRW:
        if (o.i0 == 0) {
          const Shape& sh = c.descs[o.desc].sh;
          const double cols = sh.dims[o.axis], rows = sh.size / cols;
          f = 16.0 * rows * cols * cols;
        }
        break;
      case OP_BOND: {
        const BondDesc& b = c.bonds[o.desc];
        const double Du = b.Du, Dv = b.Dv;
        f = 8.0 * c.opts.krylov_dim * (Du * Du * Dv + Du * Dv * Dv) * (1 + b.n_pairs);
        break;
      }
      default:
        break;
    }
    c.step_flops[o.tree] += f;
    c.heff_flops[o.tree] += fh;
  }
  c.step_ops = persistent_prog;  // the wide executor runs the trees one after another
  c.tree_prog = persistent_prog;
  c.scratch_desc = (int)c.descs.size();
  c.descs.resize(c.descs.size() + kScratchDescs);
  auto take = [&](size_t b) {
    size_t r = align256(off);
    off = r + std::max<size_t>(b, 1);
    return r;
  };
  c.o_descs = take(c.descs.size() * sizeof(ApplyDesc));
  c.o_modes = take(c.modes.size() * sizeof(ModeDesc));
  c.o_bonds = take(c.bonds.size() * sizeof(BondDesc));
  c.o_trees = take(c.trees.size() * sizeof(TreeDev));
  // the op table is read by the persistent executor
  c.o_prog = take(c.persistent ? persistent_prog.size() * sizeof(Op) : 0);
  c.o_begin = take(c.trees.size() * sizeof(int));
  c.o_end = take(c.trees.size() * sizeof(int));
  c.total = align256(off);
  {
    int vrc = validate_program(c, init_ops, false);
    if (!vrc) vrc = validate_program(c, persistent_prog, false);
    if (vrc) return vrc;
  }
  if (size_only) {
    *bytes_out = c.total;
    return TTNS_OK;
  }
  if (ws_bytes < c.total)
    return fail(TTNS_ENOMEM, "workspace too small: need " + std::to_string(c.total) + " bytes");
  c.ws_bytes = ws_bytes;
  c.stream = (hipStream_t)stream;
  if (!c.noalloc) HIPCHK(hipStreamCreateWithFlags(&c.cap, hipStreamNonBlocking));
  c.tables.descs = (const ApplyDesc*)(c.ws + c.o_descs);
  c.tables.modes = (const ModeDesc*)(c.ws + c.o_modes);
  c.tables.bonds = (const BondDesc*)(c.ws + c.o_bonds);
  c.tables.trees = (const TreeDev*)(c.ws + c.o_trees);
  c.d_ops = (Op*)(c.ws + c.o_prog);
  c.d_begin = (int*)(c.ws + c.o_begin);
  c.d_end = (int*)(c.ws + c.o_end);
  // zero the workspace once (environments, scalars, counters, records)
  HIPCHK(hipMemsetAsync(c.ws, 0, c.total, c.stream));
  int rc;
  for (auto& t : c.trees) {
    for (size_t k = 0; k < t.ht.ops.size(); ++k)
      if ((rc = upload(c, t.o_opdata[k], t.ht.ops[k].data(), t.ht.ops[k].size() * sizeof(cd)))) return rc;
    for (int v = 0; v < t.n; ++v)
      if (!t.site[v].empty())
        if ((rc = upload(c, t.o_sitedata[v], t.site[v].data(), t.site[v].size() * sizeof(cd)))) return rc;
    // initial tensors: the root centre init(0) (x) children's first states,
    // and column 0 of every other node's isometry, init(v) (x) first states;
    // the device QR below completes the isometries
    for (int v = 0; v < t.n; ++v) {
      const Shape& sh = t.shape[v];
      std::vector<cd> x((size_t)sh.size, cd{0, 0});
      for (int s = 0; s < sh.dims[sh.phys_axis]; ++s) x[(size_t)s * sh.stride[sh.phys_axis]] = t.ht.init[v][s];
      if ((rc = upload(c, t.o_T[v], x.data(), x.size() * sizeof(cd)))) return rc;
    }
  }
  std::vector<TreeDev> tdev;
  for (auto& t : c.trees) tdev.push_back(t.dev);
  if ((rc = upload(c, c.o_descs, c.descs.data(), c.descs.size() * sizeof(ApplyDesc)))) return rc;
  if ((rc = upload(c, c.o_modes, c.modes.data(), c.modes.size() * sizeof(ModeDesc)))) return rc;
  if ((rc = upload(c, c.o_bonds, c.bonds.data(), c.bonds.size() * sizeof(BondDesc)))) return rc;
  if ((rc = upload(c, c.o_trees, tdev.data(), tdev.size() * sizeof(TreeDev)))) return rc;
  if (c.persistent)
    if ((rc = upload(c, c.o_prog, persistent_prog.data(), persistent_prog.size() * sizeof(Op)))) return rc;
  if ((rc = upload(c, c.o_begin, c.tree_begin.data(), c.tree_begin.size() * sizeof(int)))) return rc;
  if ((rc = upload(c, c.o_end, c.tree_end.data(), c.tree_end.size() * sizeof(int)))) return rc;
  if ((rc = set_half(c, 0.0))) return rc;
  if ((rc = run_ops(c, init_ops))) return rc;
  HIPCHK(hipStreamSynchronize(c.stream));
  return TTNS_OK;
}

// Every pointer a descriptor or an op hands to a kernel must lie inside the
// workspace with the extent the kernel will touch (checked on the host
// before the first launch; a failure is an internal error, not a launch).
struct RangeCheck {
  const char* lo;
  const char* hi;
  std::string err;
  bool in(const void* p, size_t bytes, const char* what) {
    const char* q = (const char*)p;
    if (!q || q < lo || q + bytes > hi) {
      if (err.empty()) err = std::string("internal: ") + what + " outside the workspace";
      return false;
    }
    return true;
  }
};

bool check_desc(RangeCheck& rc, const ApplyDesc& d, bool allow_user_xy) {
  const size_t n = (size_t)d.sh.size * sizeof(cd);
  if (!allow_user_xy) {
    rc.in(d.x, n, "apply input");
    rc.in(d.y, n, "apply output");
  }
  const int dp = d.sh.dims[d.sh.phys_axis];
  if (d.site) rc.in(d.site, (size_t)dp * dp * sizeof(cd), "on-site operator");
  for (int k = 0; k < d.n_entries; ++k) {
    const Entry& e = d.e[k];
    if (e.axis < 0 || e.axis >= d.sh.rank || e.axis == d.sh.phys_axis) {
      rc.err = "internal: entry axis";
      return false;
    }
    const int D = d.sh.dims[e.axis];
    rc.in(e.E, (size_t)D * D * sizeof(cd), "environment channel");
    if (e.op) rc.in(e.op, (size_t)dp * dp * sizeof(cd), "entry operator");
    if (e.src >= 0 && (e.src >= kMaxTmp || !rc.in(d.tmp[e.src], n, "temporary"))) return false;
  }
  return rc.err.empty();
}

int validate_program(ttns_ctx& c, const std::vector<Op>& ops, bool allow_user_xy) {
  RangeCheck rc{c.ws, c.ws + c.total, {}};
  for (const Op& o : ops) {
    const TreeState& t = c.trees[o.tree];
    const TreeDev& d = t.dev;
    const size_t C = sizeof(cd);
    switch (o.type) {
      case OP_APPLY:
      case OP_APPLY_LZ: {
        const ApplyDesc& a = c.descs[o.desc];
        const bool user = o.desc >= c.scratch_desc;
        check_desc(rc, a, user || o.p0 != nullptr);
        if (o.p0) rc.in(o.p0, (size_t)a.sh.size * C, "apply input override");
        if (o.i1 < 0 || o.i1 > 3 || (o.type == OP_APPLY_LZ && o.i0 && o.i1))
          rc.err = "internal: apply lanes per element";
        else if ((((size_t)o.nvb * kBlock) >> o.i1) < (size_t)a.sh.size)
          rc.err = "internal: apply grid too small";
        if (o.type == OP_APPLY_LZ && (o.j < 0 || o.j >= d.kmax || a.sh.size > d.ldv))
          rc.err = "internal: Lanczos index";
        if (o.nvb > t.max_nvb) rc.err = "internal: partial-sum slots";
        if (o.type == OP_APPLY_LZ) rc.in(o.p1, (size_t)o.nvb * kRedStride * C, "Lanczos partials");
        break;
      }
      case OP_NORM:
      case OP_SCALE:
      case OP_DOT:
        rc.in(o.p0, (size_t)o.n * C, "vector");
        if (o.type == OP_DOT) rc.in(o.p2, (size_t)o.n * C, "vector");
        if (o.n > d.ldv || o.nvb * kBlock < o.n || o.nvb > t.max_nvb) rc.err = "internal: vector op size";
        break;
      case OP_ORTH1:
      case OP_ORTH2:
      case OP_COMBINE:
        if (o.n > d.ldv || o.nvb * kBlock < o.n || o.nvb > t.max_nvb) rc.err = "internal: vector op size";
        if (o.type == OP_COMBINE) rc.in(o.p1, (size_t)o.n * C, "combine output");
        if (o.type == OP_ORTH1 || o.type == OP_ORTH2) {
          if (o.j < 0 || o.j >= d.kmax || o.i0 < 1 || o.i0 > t.max_nvb) rc.err = "internal: Lanczos fold";
          else rc.in(o.p2, (size_t)o.i0 * kRedStride * C, "Lanczos partials");
          if (o.type == OP_ORTH1) rc.in(o.p1, (size_t)o.nvb * kRedStride * C, "Lanczos partials");
        }
        break;
      case OP_COPY:
        rc.in(o.p0, (size_t)o.n * C, "copy source");
        rc.in(o.p1, (size_t)o.n * C, "copy target");
        break;
      case OP_QR: {
        const Shape& sh = c.descs[o.desc].sh;
        const int cols = sh.dims[o.axis], rows = sh.size / cols;
        rc.in(o.p1, (size_t)sh.size * C, "QR tensor");
        if (o.nvb != 1 || cols > 64 || rows < cols || rows > d.max_rows || sh.size > d.ldv ||
            o.axis == sh.phys_axis || o.i1 < 0 || o.i1 > 1 || (o.i1 == 1 && !qr_fast_fits(rows, cols)))
          rc.err = "internal: QR shape";
        break;
      }
      case OP_MODE: {
        const ModeDesc& m = c.modes[o.desc];
        const size_t n = (size_t)m.sh.size * C;
        if (!allow_user_xy || !o.p0) rc.in(o.p0 ? o.p0 : m.src, n, "matrix-core source");
        if (!allow_user_xy || !o.p1) rc.in(o.p1 ? o.p1 : m.y, n, "matrix-core output");
        const int dp = m.sh.dims[m.sh.phys_axis], D = m.sh.dims[m.axis];
        if (m.site) rc.in(m.site, (size_t)dp * dp * C, "on-site operator");
        for (int e = 0; e < m.n_e; ++e) {
          rc.in(m.E[e], (size_t)D * D * C, "environment channel");
          if (m.op[e]) rc.in(m.op[e], (size_t)dp * dp * C, "entry operator");
        }
        if (m.axis == m.sh.phys_axis || D > mode_max_bond(m.prec) || o.n != m.n_rest ||
            o.axis != dp || o.i0 != m.prec || m.n_e < 1 || m.n_e > kMaxGroup ||
            o.j != mode_padded(m.prec, D) || (o.i1 & ~7) != 0 || (o.i1 & 3) == 3 ||
            ((o.i1 & 3) == 1 && o.j > mode_small_dp(m.prec)))
          rc.err = "internal: matrix-core group";
        break;
      }
      case OP_QRW: {
        const Shape& sh = c.descs[o.desc].sh;
        const int cols = sh.dims[o.axis], rows = sh.size / cols;
        rc.in(o.p1, (size_t)sh.size * C, "QR tensor");
        if (o.nvb < 1 || o.nvb > kMaxQrVb || cols > 64 || rows < cols || rows > d.max_rows ||
            sh.size > d.ldv || o.axis == sh.phys_axis || o.i0 < 0 || o.i0 > 6 || o.j < 0 || o.j >= cols)
          rc.err = "internal: wide QR shape";
        break;
      }
      case OP_CONTRACT: {
        const Shape& sh = c.descs[o.desc].sh;
        const int D = sh.dims[o.axis];
        rc.in(o.p0, (size_t)sh.size * C, "contraction Q");
        rc.in(o.p2, (size_t)sh.size * C, "contraction Z");
        if (o.i0 == 0) rc.in(o.p1, (size_t)D * D * C, "contraction output");
        if (o.nvb > kMaxContractVb || D > t.maxC) rc.err = "internal: contraction partials";
        break;
      }
      case OP_BOND: {
        const BondDesc& b = c.bonds[o.desc];
        rc.in(b.R, (size_t)b.Du * b.Dv * C, "bond matrix");
        rc.in(b.Eu, (size_t)b.Du * b.Du * C, "bond Eu");
        rc.in(b.Ev, (size_t)b.Dv * b.Dv * C, "bond Ev");
        for (int k = 0; k < b.n_pairs; ++k) {
          rc.in(b.Euk[k], (size_t)b.Du * b.Du * C, "bond Euk");
          rc.in(b.Evk[k], (size_t)b.Dv * b.Dv * C, "bond Evk");
        }
        if (o.i0 < b.Du * b.Dv || b.Du > t.maxD || b.Dv > t.maxD || o.i1 < 0 || o.i1 > 1 ||
            (o.i1 == 1 && !bond_fast_fits(b.Du, b.Dv, d.kmax, b.n_pairs)))
          rc.err = "internal: bond size";
        break;
      }
      case OP_RECORD:
        break;
      default:
        rc.err = "internal: unknown op";
    }
    if (!rc.err.empty()) return fail(TTNS_EINVAL, rc.err);
  }
  return TTNS_OK;
}

int capture_segment(ttns_ctx& c, const Op* ops, size_t n) {
  HIPCHK(hipStreamBeginCapture(c.cap, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipSuccess;
  if (c.persistent) {
    err = launch_persistent(c.d_ops, c.d_begin, c.d_end, (int)c.trees.size(), c.tables, c.cap);
  } else {
    for (size_t i = 0; i < n && err == hipSuccess; ++i) err = launch_op(ops[i], c.tables, c.cap);
  }
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(c.cap, &g);
  if (g) c.graphs.push_back(g);
  if (err != hipSuccess) return fail(TTNS_EDEVICE, std::string("capture: ") + hipGetErrorString(err));
  if (e2 != hipSuccess) return fail(TTNS_EDEVICE, std::string("end capture: ") + hipGetErrorString(e2));
  hipGraphExec_t ge = nullptr;
  HIPCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
  c.gexecs.push_back(ge);
  return TTNS_OK;
}

int build_graph(ttns_ctx& c) {
  if (!c.gexecs.empty()) return TTNS_OK;
  int rc = TTNS_OK;
  if (c.persistent) {
    rc = capture_segment(c, nullptr, 0);
  } else {
    for (size_t i = 0; i < c.step_ops.size() && !rc; i += kGraphSegment)
      rc = capture_segment(c, c.step_ops.data() + i, std::min(kGraphSegment, c.step_ops.size() - i));
  }
  if (rc) {
    for (auto ge : c.gexecs) (void)hipGraphExecDestroy(ge);
    for (auto g : c.graphs) (void)hipGraphDestroy(g);
    c.gexecs.clear();
    c.graphs.clear();
  }
  return rc;
}

int recentre(ttns_ctx& c) {
  for (size_t ti = 0; ti < c.trees.size(); ++ti) {
    TreeState& t = c.trees[ti];
    if (t.centre == 0) continue;
    std::vector<Op> ops;
    Builder b{c, t, (int)ti, ops};
    b.move_to(0);
    int rc = validate_program(c, ops, false);
    if (!rc) rc = run_ops(c, ops);
    if (rc) return rc;
  }
  return TTNS_OK;
}

std::vector<TreeState> trees_from_api(const ttns_tree* trees, int n, std::string& err, int& rc) {
  std::vector<TreeState> out(n);
  rc = TTNS_OK;
  for (int i = 0; i < n; ++i)
    if (!api_to_tree(trees[i], out[i].ht, err)) {
      rc = TTNS_EINVAL;
      break;
    }
  return out;
}

std::vector<TreeState> trees_from_star(const ttns_star_model* m, int n, std::string& err, int& rc) {
  std::vector<TreeState> out(n);
  rc = TTNS_OK;
  for (int i = 0; i < n; ++i)
    if (!star_to_tree(m[i], out[i].ht, err)) {
      rc = TTNS_EINVAL;
      break;
    }
  return out;
}

}  // namespace

namespace ttns {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace ttns



// ====================================================== allocation-free build
// A workspace for callers that cannot allocate device memory: one static
// array per device (each device that loads the library holds it until the
// process ends), handed out to at most one live context at a time.
namespace {
constexpr size_t kNoallocBytes = (size_t)64 << 20;  // 64 MiB
constexpr int kNoallocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoallocDevices] = {};          // device address of `scratch` per device
ttns_ctx* g_noalloc_owner[kNoallocDevices] = {};    // the context using it, if any
}  // namespace

// ====================================================================== C-ABI
extern "C" {

void ttns_default_opts(ttns_opts* o) {
  if (!o) return;
  o->precision = TTNS_FP64;
  o->krylov_dim = 12;
  o->breakdown_tol = 1e-12;
  o->rank_tol = 1e-8;
  o->record_capacity = 1;
  o->executor = TTNS_EXEC_AUTO;
  o->flags = 0;
}

const char* ttns_last_error(const ttns_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

int ttns_struct_sizes(size_t* out, int32_t n) {
  if (!out || n < 1) return fail(TTNS_EINVAL, "ttns_struct_sizes: bad arguments");
  const size_t s[] = {sizeof(ttns_c64), sizeof(ttns_term), sizeof(ttns_tree), sizeof(ttns_star_model),
                      sizeof(ttns_opts), sizeof(ttnn_config)};
  for (int32_t i = 0; i < n; ++i) out[i] = i < (int32_t)(sizeof(s) / sizeof(s[0])) ? s[i] : 0;
  return TTNS_OK;
}

int ttns_ohmic_chain(double alpha, double wc, double s, int32_t L, double* c0, double* eps,
                     double* hop) {
  if (L < 1 || !c0 || !eps || (L > 1 && !hop) || !(wc > 0) || !(s > -1) || alpha < 0)
    return fail(TTNS_EINVAL, "ttns_ohmic_chain: bad arguments");
  ttns::ohmic_chain(alpha, wc, s, L, c0, eps, hop);
  return TTNS_OK;
}

int ttns_workspace_size(const ttns_tree* trees, int32_t n_trees, const ttns_opts* opts, size_t* bytes) {
  if (!trees || n_trees < 1 || !bytes) return fail(TTNS_EINVAL, "ttns_workspace_size: bad arguments");
  std::string err;
  int rc;
  auto ts = trees_from_api(trees, n_trees, err, rc);
  if (rc) return fail(rc, err);
  ttns_ctx c;
  c.tune_probe = opts && (opts->flags & TTNS_FLAG_AUTOTUNE);  // the probe plan is the larger
  return prepare(c, std::move(ts), opts, nullptr, 0, nullptr, true, bytes);
}

int ttns_star_workspace_size(const ttns_star_model* models, int32_t n, const ttns_opts* opts, size_t* bytes) {
  if (!models || n < 1 || !bytes) return fail(TTNS_EINVAL, "ttns_star_workspace_size: bad arguments");
  std::string err;
  int rc;
  auto ts = trees_from_star(models, n, err, rc);
  if (rc) return fail(rc, err);
  ttns_ctx c;
  c.tune_probe = opts && (opts->flags & TTNS_FLAG_AUTOTUNE);  // the probe plan is the larger
  return prepare(c, std::move(ts), opts, nullptr, 0, nullptr, true, bytes);
}

// Mean time of one pass of `ops` on the context's stream (after one
// untimed pass), with the range checker run first.
static int time_ops(ttns_ctx& c, const std::vector<Op>& ops, int reps, double& ms) {
  int rc = validate_program(c, ops, false);
  if (rc) return rc;
  if ((rc = run_ops(c, ops))) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  hipError_t err = hipEventRecord(e0, c.stream);
  for (int r = 0; r < reps && err == hipSuccess; ++r)
    for (const Op& o : ops) {
      err = launch_op(o, c.tables, c.stream);
      if (err != hipSuccess) break;
    }
  if (err == hipSuccess) err = hipEventRecord(e1, c.stream);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float t = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(TTNS_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(err));
  ms = t / reps;
  return TTNS_OK;
}

// The autotuner, run on a probe build whose plan holds every candidate:
// for each node class the H_eff apply of one Lanczos iteration (scalar
// gather kernel, or matrix-core groups with the small or the large tile)
// and for each tall QR shape the QR of a copy of a real node tensor (one
// workgroup, or the wide QR with 1/2, 1 and 2 times its default workgroup
// count), timed on the initial state; the fastest candidate is kept.
static int autotune(ttns_ctx& c) {
  constexpr int kReps = 5;
  char line[256];
  std::string rep;
  for (size_t ti = 0; ti < c.trees.size(); ++ti) {
    TreeState& t = c.trees[ti];
    std::vector<Op> ops;
    Builder b{c, t, (int)ti, ops};
    for (int v = 0; v < t.n; ++v) {
      if (t.mode_groups[v].empty()) continue;  // no matrix-core candidate
      std::vector<ApplyDesc> pre;
      const ApplyDesc d = b.make_sum(v, -2, t.T[v], t.dev.W, pre);
      const std::string key = b.heff_key(v, d, pre.size());
      if (c.tune_heff.count(key)) continue;
      const int n = t.shape[v].size;
      const int j = std::min(t.kmax, n) / 2;  // a mid-Lanczos iteration
      const cd* vj = t.dev.V + (size_t)j * t.dev.ldv;
      auto lz = [&](int mfma) { ops.push_back(b.lz_op(v, j, mfma != 0)); };
      double best = 0.0, ms = 0.0;
      int choice = 0, rc;
      ops.clear();
      for (int p : t.heff_pre[v]) b.apply_op(p, vj);
      lz(0);
      if ((rc = time_ops(c, ops, kReps, ms))) return rc;
      best = ms;
      snprintf(line, sizeof line, "%s: scalar %.4f ms", key.c_str(), ms);
      std::string l = line;
      bool small_fits = true;
      for (int id : t.mode_groups[v]) {
        const ModeDesc& m = c.modes[id];
        small_fits = small_fits && mode_padded(m.prec, m.sh.dims[m.axis]) <= mode_small_dp(m.prec);
      }
      auto tile_name = [](int tl) {
        return std::string((tl & 3) == 1 ? "small" : "large") + ((tl & 4) ? " tile x16" : " tile x64");
      };
      for (int tile = small_fits ? 1 : 2; tile <= 2; ++tile)
        for (int narrow = 0; narrow <= 4; narrow += 4) {
          t.mode_tile[v] = tile | narrow;
          ops.clear();
          b.mode_apply(v, vj, t.dev.W);
          lz(1);
          if ((rc = time_ops(c, ops, kReps, ms))) return rc;
          snprintf(line, sizeof line, ", matrix cores %s %.4f ms", tile_name(tile | narrow).c_str(), ms);
          l += line;
          if (ms < best) {
            best = ms;
            choice = tile | narrow;
          }
        }
      t.mode_tile[v] = 0;
      c.tune_heff[key] = choice;
      rep += l + " -> " + (choice == 0 ? std::string("scalar") : tile_name(choice)) + "\n";
    }
  }
  // tall QR shapes of the step programs
  for (const Op& q : c.step_ops) {
    if (!(q.type == OP_QR || (q.type == OP_QRW && q.i0 == 0))) continue;
    const Shape& sh = c.descs[q.desc].sh;
    const int cols = sh.dims[q.axis], rows = sh.size / cols;
    if ((size_t)rows * (cols + 2) <= (size_t)kQrLdsEntries) continue;
    const std::string key = Builder::qr_key(rows, cols);
    if (c.tune_qr.count(key)) continue;
    TreeState& t = c.trees[q.tree];
    Op base = q;
    base.type = OP_QR;
    base.nvb = 1;
    base.i0 = 0;
    base.j = 0;
    Op cp{};
    cp.type = OP_COPY;
    cp.tree = q.tree;
    cp.desc = -1;
    cp.n = sh.size;
    cp.nvb = Builder::nvb_of(sh.size);
    cp.p0 = q.p1;
    cp.p1 = t.dev.X;
    base.p1 = t.dev.X;
    const int def = Builder::qr_wide_default(rows);
    std::vector<int> cand{0};
    for (int k : {std::max(1, def / 2), def, std::min(kMaxQrVb, 2 * def)})
      if (std::find(cand.begin(), cand.end(), k) == cand.end()) cand.push_back(k);
    double best = 0.0;
    int choice = 0;
    std::string l = key + ":";
    for (size_t i = 0; i < cand.size(); ++i) {
      std::vector<Op> ops{cp};
      if (cand[i] == 0) ops.push_back(base);
      else Builder::push_wide_qr(ops, base, cols, cand[i]);
      double ms = 0.0;
      int rc = time_ops(c, ops, 3, ms);
      if (rc) return rc;
      if (cand[i] == 0) snprintf(line, sizeof line, " one workgroup %.4f ms", ms);
      else snprintf(line, sizeof line, ", wide x%d %.4f ms", cand[i], ms);
      l += line;
      if (i == 0 || ms < best) {
        best = ms;
        choice = cand[i];
      }
    }
    c.tune_qr[key] = choice;
    rep += l + " -> " + (choice == 0 ? std::string("one workgroup") : "wide x" + std::to_string(choice)) + "\n";
  }
  HIPCHK(hipStreamSynchronize(c.stream));
  c.tune_report = rep;
  return TTNS_OK;
}

static int build_common(std::vector<TreeState>&& ts, const ttns_opts* opts, void* ws, size_t ws_bytes,
                        void* stream, ttns_ctx** out, bool noalloc = false) {
  if (!out) return fail(TTNS_EINVAL, "out is null");
  *out = nullptr;
  std::unique_ptr<ttns_ctx> c(new ttns_ctx());
  c->noalloc = noalloc;
  size_t dummy = 0;
  int rc;
  if (opts && (opts->flags & TTNS_FLAG_AUTOTUNE)) {
    // probe build with every candidate planned, measure, then the real build
    std::vector<TreeState> copy = ts;
    std::unique_ptr<ttns_ctx> probe(new ttns_ctx());
    probe->tune_probe = true;
    rc = prepare(*probe, std::move(ts), opts, ws, ws_bytes, stream, false, &dummy);
    if (!rc && !probe->persistent) rc = autotune(*probe);
    c->tune_heff = probe->tune_heff;
    c->tune_qr = probe->tune_qr;
    c->tune_report = probe->tune_report;
    (void)ttns_destroy(probe.release());
    if (rc) return rc;
    ts = std::move(copy);
  }
  rc = prepare(*c, std::move(ts), opts, ws, ws_bytes, stream, false, &dummy);
  // the step graphs are captured here, so that the first ttns_tdvp_step
  // costs what every later one does
  if (!rc && !noalloc) rc = build_graph(*c);
  if (rc) {
    if (c->cap) (void)hipStreamDestroy(c->cap);
    return rc;
  }
  *out = c.release();
  return TTNS_OK;
}

int ttns_build(const ttns_tree* trees, int32_t n_trees, const ttns_opts* opts, void* dev_ws,
               size_t ws_bytes, void* hip_stream, ttns_ctx** out) {
  if (!trees || n_trees < 1) return fail(TTNS_EINVAL, "ttns_build: no trees");
  std::string err;
  int rc;
  auto ts = trees_from_api(trees, n_trees, err, rc);
  if (rc) return fail(rc, err);
  return build_common(std::move(ts), opts, dev_ws, ws_bytes, hip_stream, out);
}

int ttns_star_build(const ttns_star_model* models, int32_t n_models, const ttns_opts* opts, void* dev_ws,
                    size_t ws_bytes, void* hip_stream, ttns_ctx** out) {
  if (!models || n_models < 1) return fail(TTNS_EINVAL, "ttns_star_build: no models");
  std::string err;
  int rc;
  auto ts = trees_from_star(models, n_models, err, rc);
  if (rc) return fail(rc, err);
  return build_common(std::move(ts), opts, dev_ws, ws_bytes, hip_stream, out);
}

static int ttns_apply_heff_impl(ttns_ctx* c, int32_t tree, int32_t node, const void* dev_in, void* dev_out) {
  if (!c || tree < 0 || tree >= (int)c->trees.size()) return fail(TTNS_EINVAL, "ttns_apply_heff: bad tree");
  TreeState& t = c->trees[tree];
  if (node < 0 || node >= t.n || !dev_in || !dev_out) return fail(TTNS_EINVAL, "ttns_apply_heff: bad node");
  std::vector<Op> ops;
  Builder b{*c, t, tree, ops};
  b.move_to(node);
  if (!t.mode_groups[node].empty()) {
    b.mode_apply(node, (const cd*)dev_in, (cd*)dev_out);
    int rc = validate_program(*c, ops, true);
    if (rc) return rc;
    return run_ops(*c, ops);
  }
  std::vector<ApplyDesc> pre;
  ApplyDesc d = b.make_sum(node, -2, (const cd*)dev_in, (cd*)dev_out, pre);
  const int s0 = c->scratch_desc;
  c->descs[s0] = d;
  for (size_t k = 0; k < pre.size(); ++k) c->descs[s0 + 1 + k] = pre[k];
  // every earlier launch on the stream has finished once this copy returns
  int rc = upload(*c, c->o_descs + (size_t)s0 * sizeof(ApplyDesc), &c->descs[s0],
                  (1 + pre.size()) * sizeof(ApplyDesc));
  if (rc) return rc;
  for (size_t k = 0; k < pre.size(); ++k) b.apply_op(s0 + 1 + (int)k);
  b.apply_op(s0);
  if ((rc = validate_program(*c, ops, true))) return rc;
  return run_ops(*c, ops);
}

static int ttns_tdvp_step_impl(ttns_ctx* c, double dt, int32_t n_steps) {
  if (!c || n_steps < 0 || !std::isfinite(dt)) return fail(TTNS_EINVAL, "ttns_tdvp_step: bad arguments");
  if (n_steps == 0) return TTNS_OK;
  int rc = recentre(*c);
  if (rc) return rc;
  rc = set_half(*c, 0.5 * dt);
  if (rc) return rc;
  if (c->profile && !c->persistent) {
    for (int s = 0; s < n_steps; ++s)
      if ((rc = run_ops(*c, c->step_ops))) return rc;
    return TTNS_OK;
  }
  if (c->noalloc) {  // no graphs: their instantiation allocates
    for (int s = 0; s < n_steps; ++s) {
      if (c->persistent)
        HIPCHK(launch_persistent(c->d_ops, c->d_begin, c->d_end, (int)c->trees.size(), c->tables, c->stream));
      else if ((rc = run_ops(*c, c->step_ops)))
        return rc;
    }
    return TTNS_OK;
  }
  if ((rc = build_graph(*c))) return rc;
  for (int s = 0; s < n_steps; ++s)
    for (auto ge : c->gexecs) HIPCHK(hipGraphLaunch(ge, c->stream));
  return TTNS_OK;
}

static int ttns_observe_impl(ttns_ctx* c, int32_t kind, int32_t tree, int32_t index, double* host_out, size_t n_out) {
  if (!c || tree < 0 || tree >= (int)c->trees.size() || !host_out)
    return fail(TTNS_EINVAL, "ttns_observe: bad arguments");
  TreeState& t = c->trees[tree];
  HIPCHK(hipStreamSynchronize(c->stream));
  if (kind != TTNS_OBS_STATS && kind != TTNS_OBS_RECORD_SIZE && kind != TTNS_OBS_BOND_DIMS &&
      kind != TTNS_OBS_STEP_FLOPS) {
    // numerical failures flagged by the kernels: bit 0 a QR that found no
    // completion vector, bit 1 a non-finite record
    int flags = 0;
    HIPCHK(hipMemcpy(&flags, t.dev.stats + 3, sizeof(int), hipMemcpyDeviceToHost));
    if (flags & 1) return fail(TTNS_ENUMERIC, "ttns_observe: a QR found no completion vector (non-finite state)");
    if (flags & 2) return fail(TTNS_ENUMERIC, "ttns_observe: a step produced a non-finite norm or density matrix");
  }
  int count = 0;
  HIPCHK(hipMemcpy(&count, t.dev.rec_count, sizeof(int), hipMemcpyDeviceToHost));
  const int rs = t.rec_size, nel = t.n_el;
  auto need = [&](size_t k) { return n_out >= k ? TTNS_OK : fail(TTNS_EINVAL, "ttns_observe: output too small"); };
  std::vector<double> rec(rs);
  auto last = [&]() -> int {
    if (count < 1) return fail(TTNS_EINVAL, "ttns_observe: nothing recorded");
    HIPCHK(hipMemcpy(rec.data(), t.dev.hist + (size_t)(count - 1) * rs, rs * sizeof(double),
                     hipMemcpyDeviceToHost));
    return TTNS_OK;
  };
  int rc;
  switch (kind) {
    case TTNS_OBS_RDM:
      if ((rc = need(2 * (size_t)nel * nel)) || (rc = last())) return rc;
      std::memcpy(host_out, rec.data(), 2 * (size_t)nel * nel * sizeof(double));
      return TTNS_OK;
    case TTNS_OBS_POP:
      if ((rc = need(nel)) || (rc = last())) return rc;
      for (int j = 0; j < nel; ++j) host_out[j] = rec[2 * (j * nel + j)];
      return TTNS_OK;
    case TTNS_OBS_NORM:
      if ((rc = need(1)) || (rc = last())) return rc;
      host_out[0] = rec[2 * nel * nel];
      return TTNS_OK;
    case TTNS_OBS_ENERGY:
      if ((rc = need(1)) || (rc = last())) return rc;
      host_out[0] = rec[2 * nel * nel + 1];
      return TTNS_OK;
    case TTNS_OBS_LOCAL: {
      const size_t no = t.ht.obs_node.size();
      if ((rc = need(no)) || (rc = last())) return rc;
      for (size_t k = 0; k < no; ++k) host_out[k] = rec[2 * nel * nel + 2 + k];
      return TTNS_OK;
    }
    case TTNS_OBS_HISTORY:
      if ((rc = need((size_t)count * rs))) return rc;
      HIPCHK(hipMemcpy(host_out, t.dev.hist, (size_t)count * rs * sizeof(double), hipMemcpyDeviceToHost));
      return TTNS_OK;
    case TTNS_OBS_RECORD_SIZE:
      if ((rc = need(1))) return rc;
      host_out[0] = rs;
      return TTNS_OK;
    case TTNS_OBS_TENSOR: {
      if (index < 0 || index >= t.n) return fail(TTNS_EINVAL, "ttns_observe: bad node");
      const size_t n = 2 * (size_t)t.shape[index].size;
      if ((rc = need(n))) return rc;
      HIPCHK(hipMemcpy(host_out, t.T[index], n * sizeof(double), hipMemcpyDeviceToHost));
      return TTNS_OK;
    }
    case TTNS_OBS_STATS: {
      if ((rc = need(5))) return rc;
      int st[8];
      HIPCHK(hipMemcpy(st, t.dev.stats, sizeof(st), hipMemcpyDeviceToHost));
      host_out[0] = count;
      host_out[1] = st[0];
      host_out[2] = st[2];
      host_out[3] = st[1];
      host_out[4] = st[3];
      return TTNS_OK;
    }
    case TTNS_OBS_STEP_FLOPS:
      if ((rc = need(2))) return rc;
      host_out[0] = c->step_flops[tree];
      host_out[1] = c->heff_flops[tree];
      return TTNS_OK;
    case TTNS_OBS_BOND_DIMS:
      if ((rc = need(t.n))) return rc;
      for (int v = 0; v < t.n; ++v) host_out[v] = t.D[v];
      return TTNS_OK;
    case TTNS_OBS_ENTROPY: {
      if (index < 1 || index >= t.n) return fail(TTNS_EINVAL, "ttns_observe: entropy needs a non-root node");
      if ((rc = need(1))) return rc;
      // centre to `index`, then the gauge move to its parent: the QR's R
      // carries the Schmidt values of the bond
      const int par = parent_of(t, index);
      std::vector<Op> ops;
      Builder b{*c, t, tree, ops};
      b.move_to(index);
      b.move(index, par, false);
      if ((rc = validate_program(*c, ops, false)) || (rc = run_ops(*c, ops))) return rc;
      // eigenvalues of R^H R (the squared Schmidt values) and -sum p ln p
      const int D = t.shape[index].dims[axis_of(t, index, par)];
      cd* G = (cd*)(c->ws + c->o_aux);
      double* ev = (double*)(G + 2 * kAuxMat);
      HIPCHK(launch_gram(t.dev.R, D, G, c->stream));
      HIPCHK(launch_herm_eig(G, D, D, ev, nullptr, 1, c->stream));
      HIPCHK(launch_entropy(ev, D, ev + 128, c->stream));
      HIPCHK(hipMemcpyAsync(host_out, ev + 128, sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      return TTNS_OK;
    }
    default:
      return fail(TTNS_EINVAL, "ttns_observe: unknown kind");
  }
}

static int ttns_profile_impl(ttns_ctx* c, int32_t enable) {
  if (!c) return fail(TTNS_EINVAL, "ttns_profile: null context");
  c->profile = enable != 0;
  return TTNS_OK;
}

static int ttns_profile_read_impl(ttns_ctx* c, int32_t reset, double* avg_ms, int64_t* launches, double* flops) {
  if (!c) return fail(TTNS_EINVAL, "ttns_profile_read: null context");
  int rc = drain_profile(*c);
  if (rc) return rc;
  double ms = 0.0, fl = 0.0;
  int64_t n = 0;
  for (int k : {(int)TTNS_K_HEFF_LZ, (int)TTNS_K_MODE_FP64, (int)TTNS_K_MODE_FP32, (int)TTNS_K_MODE_BF16X3}) {
    ms += c->cls_ms[k];
    fl += c->cls_flops[k];
    n += c->cls_n[k];
  }
  if (avg_ms) *avg_ms = n ? ms / n : 0.0;
  if (launches) *launches = n;
  if (flops) *flops = n ? fl / n : 0.0;
  if (reset)
    for (int i = 0; i < TTNS_K_COUNT; ++i) {
      c->cls_ms[i] = c->cls_flops[i] = c->cls_bytes[i] = 0.0;
      c->cls_n[i] = 0;
    }
  return TTNS_OK;
}

static int ttns_profile_kernel_impl(ttns_ctx* c, int32_t kernel, double* total_ms, int64_t* launches, double* flops,
                        double* bytes) {
  if (!c || kernel < 0 || kernel >= TTNS_K_COUNT) return fail(TTNS_EINVAL, "ttns_profile_kernel: bad arguments");
  int rc = drain_profile(*c);
  if (rc) return rc;
  if (total_ms) *total_ms = c->cls_ms[kernel];
  if (launches) *launches = c->cls_n[kernel];
  if (flops) *flops = c->cls_flops[kernel];
  if (bytes) *bytes = c->cls_bytes[kernel];
  return TTNS_OK;
}

int ttns_tuning_report(const ttns_ctx* c, char* out, size_t n, size_t* needed) {
  if (!c || (!out && n > 0)) return fail(TTNS_EINVAL, "ttns_tuning_report: bad arguments");
  if (needed) *needed = c->tune_report.size() + 1;
  if (n > 0) {
    const size_t k = std::min(n - 1, c->tune_report.size());
    memcpy(out, c->tune_report.data(), k);
    out[k] = 0;
  }
  return TTNS_OK;
}

// Energy surfaces (Eqs. 3-4): bath Schmidt states of the root, the matrix of
// the context's operator sum between (bath state, electronic state)
// products, its eigenvalues.
static int ttns_energy_surfaces_impl(ttns_ctx* c, int32_t tree, double rank_tol, int32_t* n_bath,
                                     double* host_values, double* host_matrix, size_t cap) {
  if (!c || tree < 0 || tree >= (int)c->trees.size() || !host_values || !n_bath || !(rank_tol > 0) ||
      !(rank_tol < 1))
    return fail(TTNS_EINVAL, "ttns_energy_surfaces: bad arguments");
  TreeState& t = c->trees[tree];
  const int nel = t.n_el, size = t.shape[0].size, nb = size / nel;
  if (nel > 8 || nel * nel > surf_eig_max())
    return fail(TTNS_EINVAL, "ttns_energy_surfaces: at most 8 electronic levels");
  if ((size_t)nel * nel > cap) return fail(TTNS_EINVAL, "ttns_energy_surfaces: host_values holds fewer than n^2 values");
  if (2 * nel > t.kmax + 1) return fail(TTNS_EINVAL, "ttns_energy_surfaces: Krylov basis too small for the bath states");
  int rc = recentre(*c);
  if (rc) return rc;
  cd* M = (cd*)(c->ws + c->o_aux);
  cd* Wv = M + kAuxMat;
  double* ev = (double*)(Wv + kAuxMat);
  cd* part = (cd*)(ev + 256);
  // rho^T = conj(rho) of the root (the contraction over all bonds)
  {
    std::vector<Op> ops;
    Builder b{*c, t, tree, ops};
    Op o = b.base(OP_CONTRACT, std::min(kMaxContractVb, std::max(1, (nb + 31) / 32)));
    o.desc = t.heff_desc[0];
    o.axis = 0;
    o.p0 = t.T[0];
    o.p2 = t.T[0];
    o.p1 = M;
    o.i0 = 0;
    ops.push_back(o);
    if ((rc = validate_program_aux(*c, ops))) return rc;
    if ((rc = run_ops(*c, ops))) return rc;
  }
  // Schmidt decomposition C = U S Vh in two passes: the eigenvectors of rho
  // rotate the rows of C to nearly orthogonal ones (U^H C), whose own Gram
  // matrix is then graded (diagonal s_i^2), so a second eigen-decomposition
  // gets the small singular values' directions to rounding relative to
  // their size (rho alone would leave them at rounding relative to s_0)
  const int nvb = std::min(kSurfVb, std::max(1, (nb + 1023) / 1024));
  cd* Bm = t.dev.V;                            // rows U^H C: Krylov rows [0, n)
  cd* B = t.dev.V + (size_t)nel * t.dev.ldv;   // bath states: rows [n, 2n)
  HIPCHK(launch_herm_eig(M, nel, nel, ev, Wv, 1, c->stream));
  HIPCHK(launch_bath_vectors(t.T[0], nb, nel, nb, Wv, ev, nel, 0, Bm, t.dev.ldv, c->stream));
  HIPCHK(launch_surf_dots(Bm, t.dev.ldv, Bm, t.dev.ldv, nel, nb, nel, part, nvb, c->stream));
  HIPCHK(launch_surf_fold(part, nvb, nel * nel, M, 1, 0, c->stream));
  HIPCHK(launch_herm_eig(M, nel, nel, ev, Wv, 1, c->stream));
  std::vector<double> lam(nel);
  HIPCHK(hipMemcpyAsync(lam.data(), ev, nel * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  // retained bath states: s_i > rank_tol s_0, i.e. lambda_i > rank_tol^2 lambda_0
  int r = 0;
  for (int i = nel - 1; i >= 0; --i)
    if (lam[i] > rank_tol * rank_tol * lam[nel - 1] && lam[i] > 0.0) ++r;
  if (r == 0) return fail(TTNS_ENUMERIC, "ttns_energy_surfaces: the state is zero");
  *n_bath = r;
  const int N = r * nel;
  HIPCHK(launch_bath_vectors(Bm, t.dev.ldv, nel, nb, Wv, ev, r, 1, B, t.dev.ldv, c->stream));
  for (int k = 0; k < r; ++k)
    for (int l = 0; l < nel; ++l) {
      HIPCHK(launch_surf_fill(t.dev.X, B, t.dev.ldv, k, l, nel, nb, c->stream));
      std::vector<Op> ops;
      Builder b{*c, t, tree, ops};
      if (!t.mode_groups[0].empty()) {
        b.mode_apply(0, t.dev.X, t.dev.W);
      } else {
        for (int pid : t.heff_pre[0]) b.apply_op(pid, t.dev.X);
        b.apply_op(t.heff_desc[0], t.dev.X);  // y = W
      }
      if ((rc = validate_program_aux(*c, ops))) return rc;
      if ((rc = run_ops(*c, ops))) return rc;
      HIPCHK(launch_surf_dots(B, t.dev.ldv, t.dev.W, nb, nel, nb, r, part, nvb, c->stream));
      HIPCHK(launch_surf_fold(part, nvb, N, M, N, k * nel + l, c->stream));
    }
  HIPCHK(launch_herm_eig(M, N, N, ev, nullptr, 0, c->stream));
  HIPCHK(hipMemcpyAsync(host_values, ev, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (host_matrix)
    HIPCHK(hipMemcpyAsync(host_matrix, M, (size_t)N * N * sizeof(cd), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return TTNS_OK;
}

// dst's tree takes src's state (same shapes), centre at the root, and
// rebuilds its environments towards the root for its own operator sum.
static int ttns_copy_state_impl(ttns_ctx* dst, int32_t dtree, ttns_ctx* src, int32_t stree) {
  if (!dst || !src || dtree < 0 || dtree >= (int)dst->trees.size() || stree < 0 ||
      stree >= (int)src->trees.size())
    return fail(TTNS_EINVAL, "ttns_copy_state: bad arguments");
  TreeState& td = dst->trees[dtree];
  TreeState& ts = src->trees[stree];
  if (td.n != ts.n || td.ht.parent != ts.ht.parent)
    return fail(TTNS_EINVAL, "ttns_copy_state: the trees differ");
  for (int v = 0; v < td.n; ++v)
    for (int a = 0; a < kMaxRank; ++a)
      if (td.shape[v].dims[a] != ts.shape[v].dims[a])
        return fail(TTNS_EINVAL, "ttns_copy_state: node " + std::to_string(v) + " has another shape");
  int rc = recentre(*src);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(src->stream));
  for (int v = 0; v < td.n; ++v)
    HIPCHK(hipMemcpyAsync(td.T[v], ts.T[v], (size_t)td.shape[v].size * sizeof(cd), hipMemcpyDeviceToDevice,
                          dst->stream));
  std::vector<Op> ops;
  Builder b{*dst, td, dtree, ops};
  for (int v = td.n - 1; v > 0; --v) b.env_update(v, parent_of(td, v));
  if ((rc = validate_program(*dst, ops, false))) return rc;
  if ((rc = run_ops(*dst, ops))) return rc;
  td.centre = 0;
  HIPCHK(hipStreamSynchronize(dst->stream));
  return TTNS_OK;
}

// Entry points on a context: the message of a failure is kept on the
// context as well as for the calling thread.
#define TTNS_CTX_CALL(c, expr)            \
  do {                                    \
    const int rc_ = (expr);               \
    if (rc_ != TTNS_OK && (c)) (c)->err = g_err; \
    return rc_;                           \
  } while (0)

int ttns_apply_heff(ttns_ctx* c, int32_t tree, int32_t node, const void* dev_in, void* dev_out) {
  TTNS_CTX_CALL(c, ttns_apply_heff_impl(c, tree, node, dev_in, dev_out));
}
int ttns_tdvp_step(ttns_ctx* c, double dt, int32_t n_steps) { TTNS_CTX_CALL(c, ttns_tdvp_step_impl(c, dt, n_steps)); }
int ttns_observe(ttns_ctx* c, int32_t kind, int32_t tree, int32_t index, double* host_out, size_t n_out) {
  TTNS_CTX_CALL(c, ttns_observe_impl(c, kind, tree, index, host_out, n_out));
}
int ttns_profile(ttns_ctx* c, int32_t enable) { TTNS_CTX_CALL(c, ttns_profile_impl(c, enable)); }
int ttns_energy_surfaces(ttns_ctx* c, int32_t tree, double rank_tol, int32_t* n_bath, double* host_values,
                         double* host_matrix, size_t cap) {
  TTNS_CTX_CALL(c, ttns_energy_surfaces_impl(c, tree, rank_tol, n_bath, host_values, host_matrix, cap));
}
int ttns_copy_state(ttns_ctx* dst, int32_t dst_tree, ttns_ctx* src, int32_t src_tree) {
  TTNS_CTX_CALL(dst, ttns_copy_state_impl(dst, dst_tree, src, src_tree));
}
int ttns_profile_read(ttns_ctx* c, int32_t reset, double* avg_ms, int64_t* launches, double* flops) {
  TTNS_CTX_CALL(c, ttns_profile_read_impl(c, reset, avg_ms, launches, flops));
}
int ttns_profile_kernel(ttns_ctx* c, int32_t kernel, double* total_ms, int64_t* launches, double* flops,
                        double* bytes) {
  TTNS_CTX_CALL(c, ttns_profile_kernel_impl(c, kernel, total_ms, launches, flops, bytes));
}

int ttns_destroy(ttns_ctx* c) {
  if (!c) return TTNS_OK;
  if (c->noalloc && c->noalloc_dev >= 0) {
    (void)hipStreamSynchronize(c->stream);  // the next owner may clear the array
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_owner[c->noalloc_dev] == c) g_noalloc_owner[c->noalloc_dev] = nullptr;
  }
  drain_profile(*c);
  for (auto ge : c->gexecs) (void)hipGraphExecDestroy(ge);
  for (auto g : c->graphs) (void)hipGraphDestroy(g);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
  return TTNS_OK;
}

}  // extern "C"

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

extern "C" int ttns_star_build_noalloc(const ttns_star_model* models, int32_t n_models, const ttns_opts* opts,
                                       void* hip_stream, ttns_ctx** out) {
  if (!out) return fail(TTNS_EINVAL, "ttns_star_build_noalloc: out is null");
  *out = nullptr;
  if (!models || n_models < 1) return fail(TTNS_EINVAL, "ttns_star_build_noalloc: no models");
  if (opts && (opts->flags & TTNS_FLAG_AUTOTUNE))
    return fail(TTNS_EINVAL, "ttns_star_build_noalloc: the autotuner's timing events allocate; build without it");
  size_t need = 0;
  int rc = ttns_star_workspace_size(models, n_models, opts, &need);
  if (rc) return rc;
  if (need > kNoallocBytes)
    return fail(TTNS_ENOMEM, "ttns_star_build_noalloc: the trees need " + std::to_string(need) +
                                 " bytes of workspace, the static workspace holds " + std::to_string(kNoallocBytes));
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoallocDevices) return fail(TTNS_EDEVICE, "ttns_star_build_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    // the array's address on this device (the host-side name is not one)
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TTNS_EDEVICE, std::string("ttns_star_build_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_noalloc_ptr[dev] = p;
  }
  if (g_noalloc_owner[dev])
    return fail(TTNS_EINVAL, "ttns_star_build_noalloc: the static workspace of device " + std::to_string(dev) +
                                 " is held by another context; destroy it first");
  std::string err;
  auto ts = trees_from_star(models, n_models, err, rc);
  if (rc) return fail(rc, err);
  rc = build_common(std::move(ts), opts, g_noalloc_ptr[dev], kNoallocBytes, hip_stream, out, true);
  if (rc) return rc;
  (*out)->noalloc_dev = dev;
  g_noalloc_owner[dev] = *out;
  return TTNS_OK;
}

