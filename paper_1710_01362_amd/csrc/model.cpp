// Model assembly on the host (FP64): the chain mapping of each bosonic
// environment and the star / ER-tree operator sum of Eq. (2), plus the
// translation of a caller-given tree (ttns_tree) into the internal form.
#include <cmath>
#include <functional>
#include <map>

#include "ttns_internal.h"

namespace ttns {

// Orthogonal-polynomial chain of J(w) = 2 pi alpha wc (w/wc)^s theta(wc - w)
// (closed-form recurrence of the shifted Jacobi polynomials, Chin et al.,
// J. Math. Phys. 51, 092109 (2010), the mapping the paper applies to every
// cluster of modes): site energies eps_n, hoppings t_n, and the system-site-0
// coupling c0 = sqrt(eta0 / pi) with eta0 = int J = 2 pi alpha wc^2 / (1+s).
void ohmic_chain(double alpha, double wc, double s, int L, double* c0,
                 double* eps, double* hop) {
  *c0 = wc * std::sqrt(2.0 * alpha / (1.0 + s));
  for (int n = 0; n < L; ++n) {
    double a = s + 2.0 * n;
    eps[n] = 0.5 * wc * (1.0 + s * s / (a * (a + 2.0)));
  }
  for (int n = 0; n + 1 < L; ++n) {
    double a = s + 2.0 * n;
    hop[n] = wc * (n + 1.0) * (n + 1.0 + s) / ((a + 2.0) * (a + 3.0)) *
             std::sqrt((a + 3.0) / (a + 1.0));
  }
}

namespace {

int add_op(HostTree& t, const std::vector<cd>& m, int d) {
  t.ops.push_back(m);
  t.opdim.push_back(d);
  return (int)t.ops.size() - 1;
}

int add_node(HostTree& t, int parent, int d, int D, const std::vector<cd>& loc) {
  t.parent.push_back(parent);
  t.phys.push_back(d);
  t.bondreq.push_back(D);
  t.init.push_back(loc);
  return t.n++;
}

struct BosonOps {
  int b, bd, num, x, p, p2;  // p = i (b^+ - b) / sqrt(2), p2 = p p
};

BosonOps boson_ops(HostTree& t, int d, std::map<int, BosonOps>& cache) {
  auto it = cache.find(d);
  if (it != cache.end()) return it->second;
  std::vector<cd> b(d * d, cd{0, 0}), bd(d * d, cd{0, 0}), num(d * d, cd{0, 0}),
      x(d * d, cd{0, 0});
  for (int k = 1; k < d; ++k) {
    double v = std::sqrt((double)k);
    b[(k - 1) * d + k] = cd{v, 0};   // b|k> = sqrt(k)|k-1>
    bd[k * d + (k - 1)] = cd{v, 0};
    x[(k - 1) * d + k] = cd{v, 0};
    x[k * d + (k - 1)] = cd{v, 0};
  }
  for (int k = 0; k < d; ++k) num[k * d + k] = cd{(double)k, 0};
  // momentum p = i (b^+ - b) / sqrt(2) and its square (matrix product in the
  // truncated space)
  std::vector<cd> pm(d * d, cd{0, 0}), p2(d * d, cd{0, 0});
  const double r2 = 1.0 / std::sqrt(2.0);
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      const double v = bd[r * d + c].x - b[r * d + c].x;  // real
      pm[r * d + c] = cd{0.0, v * r2};
    }
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      double re = 0.0, im = 0.0;
      for (int k = 0; k < d; ++k) {
        const cd a = pm[r * d + k], e = pm[k * d + c];
        re += a.x * e.x - a.y * e.y;
        im += a.x * e.y + a.y * e.x;
      }
      p2[r * d + c] = cd{re, im};
    }
  BosonOps o{add_op(t, b, d), add_op(t, bd, d), add_op(t, num, d), add_op(t, x, d), add_op(t, pm, d),
             add_op(t, p2, d)};
  cache[d] = o;
  return o;
}

}  // namespace

bool star_to_tree(const ttns_star_model& m, HostTree& t, std::string& err) {
  const int n = m.n_levels;
  if (n < 1 || !m.h_el || !m.init_el || m.n_chains < 0) {
    err = "star model: bad electronic part";
    return false;
  }
  if (m.n_chains > 0 && (!m.coupling || !m.alpha || !m.wc || !m.s || !m.length ||
                         !m.local_dim || !m.bond_dim)) {
    err = "star model: missing chain arrays";
    return false;
  }
  t = HostTree();
  t.n_levels_hint = n;
  std::vector<cd> hel((size_t)n * n);
  for (int i = 0; i < n * n; ++i) hel[i] = cd{m.h_el[i].re, m.h_el[i].im};
  std::vector<cd> init(n);
  for (int i = 0; i < n; ++i) init[i] = cd{m.init_el[i].re, m.init_el[i].im};
  add_node(t, -1, n, 0, init);
  int op_hel = add_op(t, hel, n);
  t.terms.push_back(HostTerm{0, op_hel, -1, -1, 1.0});
  std::map<int, BosonOps> cache;

  auto add_chain = [&](int i, int p) -> bool {
    int L = m.length[i], d = m.local_dim[i], D = m.bond_dim[i];
    if (L < 1 || d < 1 || D < 1 || m.wc[i] <= 0 || m.alpha[i] < 0 || m.s[i] <= -1) {
      err = "star model: bad chain parameters";
      return false;
    }
    std::vector<double> eps(L), hop(L > 1 ? L - 1 : 1);
    double c0;
    ohmic_chain(m.alpha[i], m.wc[i], m.s[i], L, &c0, eps.data(), hop.data());
    BosonOps bo = boson_ops(t, d, cache);
    std::vector<cd> A(n * n);
    for (int k = 0; k < n * n; ++k)
      A[k] = cd{m.coupling[(size_t)i * n * n + k].re, m.coupling[(size_t)i * n * n + k].im};
    int op_A = add_op(t, A, n);
    std::vector<cd> vac(d, cd{0, 0});
    vac[0] = cd{1, 0};
    const int obb = m.obb_dim ? m.obb_dim[i] : 0;
    int prev = p, head = -1;
    std::vector<int> nodes;  // the nodes the boson operators act on
    std::vector<cd> unit(1, cd{1, 0});
    for (int k = 0; k < L; ++k) {
      int node;
      if (obb > 0) {
        // optimised boson basis: the site has no physical leg; its first
        // child holds the d Fock states behind a bond of dimension obb, its
        // second child is the next site
        const int site = add_node(t, prev, 1, D, unit);
        node = add_node(t, site, d, obb, vac);
        prev = site;
      } else {
        node = add_node(t, prev, d, D, vac);
        prev = node;
      }
      nodes.push_back(node);
      if (k == 0) head = node;
    }
    t.terms.push_back(HostTerm{0, op_A, head, bo.x, c0});
    for (int k = 0; k < L; ++k) t.terms.push_back(HostTerm{nodes[k], bo.num, -1, -1, eps[k]});
    for (int k = 0; k + 1 < L; ++k) {
      t.terms.push_back(HostTerm{nodes[k], bo.bd, nodes[k + 1], bo.b, hop[k]});
      t.terms.push_back(HostTerm{nodes[k], bo.b, nodes[k + 1], bo.bd, hop[k]});
    }
    if (m.potential) {
      // H - T: T = sum over the chain's modes of (w/2) P^2 = (1/2) p^T M p
      // with M the chain's tridiagonal matrix (eps on the diagonal, hop
      // beside it) and p the site momenta
      for (int k = 0; k < L; ++k) t.terms.push_back(HostTerm{nodes[k], bo.p2, -1, -1, -0.5 * eps[k]});
      for (int k = 0; k + 1 < L; ++k) t.terms.push_back(HostTerm{nodes[k], bo.p, nodes[k + 1], bo.p, -hop[k]});
    }
    t.obs_node.push_back(head);
    t.obs_op.push_back(bo.num);
    return true;
  };

  std::vector<int> order(m.n_chains);
  for (int i = 0; i < m.n_chains; ++i) order[i] = i;
  std::vector<cd> one(1, cd{1, 0});
  // ER tree: every group of more than one chain hangs below one ER node whose
  // two children carry the two halves of the group (first half rounded up).
  std::function<bool(int, int, int)> group = [&](int p, int lo, int hi) -> bool {
    if (hi - lo == 1) return add_chain(order[lo], p);
    int e = add_node(t, p, 1, m.er_bond_dim, one);
    int half = (hi - lo + 1) / 2;
    return group(e, lo, lo + half) && group(e, lo + half, hi);
  };
  if (m.topology == 0 || m.n_chains <= 1) {
    for (int i = 0; i < m.n_chains; ++i)
      if (!add_chain(i, 0)) return false;
  } else if (m.topology == 1) {
    if (m.er_bond_dim < 1) {
      err = "star model: er_bond_dim must be >= 1";
      return false;
    }
    int half = (m.n_chains + 1) / 2;
    if (!group(0, 0, half) || !group(0, half, m.n_chains)) return false;
  } else {
    err = "star model: unknown topology";
    return false;
  }
  return true;
}

bool api_to_tree(const ttns_tree& a, HostTree& t, std::string& err) {
  t = HostTree();
  if (a.n_nodes < 1 || !a.parent || !a.phys_dim || !a.bond_dim || !a.init_local) {
    err = "tree: missing arrays";
    return false;
  }
  t.n = a.n_nodes;
  t.parent.assign(a.parent, a.parent + a.n_nodes);
  t.phys.assign(a.phys_dim, a.phys_dim + a.n_nodes);
  t.bondreq.assign(a.bond_dim, a.bond_dim + a.n_nodes);
  size_t off = 0;
  for (int v = 0; v < t.n; ++v) {
    if (t.phys[v] < 1) {
      err = "tree: phys_dim must be >= 1";
      return false;
    }
    std::vector<cd> loc(t.phys[v]);
    for (int s = 0; s < t.phys[v]; ++s) loc[s] = cd{a.init_local[off + s].re, a.init_local[off + s].im};
    off += t.phys[v];
    t.init.push_back(loc);
  }
  off = 0;
  for (int k = 0; k < a.n_ops; ++k) {
    int d = a.op_dim[k];
    if (d < 1) {
      err = "tree: op_dim must be >= 1";
      return false;
    }
    std::vector<cd> m(d * d);
    for (int i = 0; i < d * d; ++i) m[i] = cd{a.op_data[off + i].re, a.op_data[off + i].im};
    off += (size_t)d * d;
    t.ops.push_back(m);
    t.opdim.push_back(d);
  }
  for (int k = 0; k < a.n_terms; ++k) {
    const ttns_term& x = a.terms[k];
    t.terms.push_back(HostTerm{x.node_a, x.op_a, x.node_b, x.op_b, x.coef});
  }
  for (int k = 0; k < a.n_observe; ++k) {
    t.obs_node.push_back(a.observe_node[k]);
    t.obs_op.push_back(a.observe_op[k]);
  }
  return true;
}

}  // namespace ttns
