/*
 * ttns.h -- C-ABI of the MI355X tree-tensor-network-state (TTNS) one-site
 * TDVP library.
 *
 * What it computes.  The state of a system coupled to bosonic environments is
 * a TTNS (paper: "TTNS for vibronic quantum dynamics"): one tensor per tree
 * node, the electronic levels at the root, one node per chain site of the
 * chain-mapped environments of Eq. (2), optionally entanglement-
 * renormalisation (ER) nodes between the root and the chains (Fig. 2).  The
 * Hamiltonian is given as an operator sum over nodes ("tree MPO").  A time
 * step evolves every node with exp(-i h H_eff) and every bond matrix with
 * exp(+i h H_bond), sequentially over the tree, where H_eff is rebuilt from
 * the full state at every node visit (the time-dependent variational
 * principle the paper uses; Methods, "Tensor Network States").  The local
 * exponentials are Lanczos/Krylov approximations.
 *
 * Conventions.
 *   - Complex numbers are ttns_c64 {re, im} (interleaved, like C99 double
 *     complex).  Operator matrices are row-major, op[r * d + c].
 *   - Nodes are numbered in pre-order: parent[0] = -1, parent[i] < i, and the
 *     nodes of every subtree are contiguous.  Children are ordered by index.
 *   - Node tensor axes: [bond to parent] (absent at the root), physical leg,
 *     bonds to the children in child order; row-major, last axis fastest.
 *   - Every call returns a status: TTNS_OK or a negative code.  No call
 *     aborts; ttns_last_error(ctx) returns the message of the context's last
 *     failure (ttns_last_error(NULL): the calling thread's).
 *   - Device pointers ("dev_") are HIP device addresses; host pointers are
 *     ordinary memory.  The caller owns every buffer it passes; the library
 *     copies host inputs during the call and never frees caller memory.
 *   - Nothing in the library allocates device memory: all device state lives
 *     in the workspace the caller passes to ttns_build.
 */
#ifndef TTNS_H
#define TTNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define TTNS_OK 0
#define TTNS_EINVAL (-1)   /* invalid argument, topology or Hamiltonian   */
#define TTNS_ENOMEM (-2)   /* workspace too small                          */
#define TTNS_EDEVICE (-3)  /* a HIP call failed                             */
#define TTNS_ENUMERIC (-4) /* non-finite values: at build, in the inputs; at
                              run time, a non-finite record (norm, energy,
                              density matrix) or a QR that found no
                              completion vector, reported by the next
                              ttns_observe of that tree                    */

/* arithmetic of the H_eff contractions (Lanczos, exponentials, QR and the
 * environments always run in FP64) */
#define TTNS_FP64 0
#define TTNS_FP32 1    /* contractions in FP32 with FP32 accumulation      */
#define TTNS_BF16X3 2  /* split-BF16 (hi*hi + hi*lo + lo*hi), FP32 accum.  */

/* executors */
#define TTNS_EXEC_AUTO 0
#define TTNS_EXEC_WIDE 1       /* each operation spread over many workgroups */
#define TTNS_EXEC_PERSISTENT 2 /* one workgroup runs a whole tree's step     */

/* option flags */
#define TTNS_FLAG_MFMA_ALL 1u  /* matrix-core H_eff for every node whose bonds
                                  fit the tiles; by default only nodes of at
                                  least 16384 entries use it (smaller ones are
                                  latency-bound and keep the scalar FP64 apply) */
#define TTNS_FLAG_AUTOTUNE 2u  /* wide executor: at build, time the H_eff
                                  variants of every node class (scalar apply,
                                  matrix-core small or large tile) and the QR
                                  variants of every tall QR shape (one
                                  workgroup, or 1/2x, 1x, 2x the default
                                  workgroup count) on the initial state, and
                                  plan the step with the fastest of each;
                                  ttns_tuning_report lists the choices.  The
                                  build then runs the initial programs twice. */

/* observables (ttns_observe kinds) */
#define TTNS_OBS_RDM 0       /* root reduced density matrix, n x n complex:
                                2 n^2 doubles (re, im), row-major           */
#define TTNS_OBS_POP 1       /* root populations rho_jj, n doubles           */
#define TTNS_OBS_LOCAL 2     /* recorded local expectation values (n_observe) */
#define TTNS_OBS_NORM 3      /* <psi|psi>, 1 double                          */
#define TTNS_OBS_ENERGY 4    /* <psi|H|psi>, 1 double                        */
#define TTNS_OBS_HISTORY 5   /* every record so far: records x record_size   */
#define TTNS_OBS_RECORD_SIZE 6 /* doubles per record (1 double)              */
#define TTNS_OBS_TENSOR 7    /* node tensor `index`, 2*size doubles          */
#define TTNS_OBS_STATS 8     /* [records, guarded QR columns, steps]          */
#define TTNS_OBS_BOND_DIMS 9 /* clamped bond dims, n_nodes doubles (0: root) */
#define TTNS_OBS_STEP_FLOPS 10 /* algorithmic real flops of one step of this
                                  tree: [total, H_eff contractions only]     */
#define TTNS_OBS_ENTROPY 11  /* von Neumann entropy -sum p ln p of the
                                Schmidt values across the bond between node
                                `index` (not the root) and its parent, i.e.
                                of the bipartition (subtree of index | rest),
                                1 double, from the current state (TTNS
                                section: S = -Tr rho ln rho of a bond),
                                computed on the device from the eigenvalues
                                of R^H R, R the bond matrix of the gauge QR.
                                It moves the centre to the parent of `index`
                                (gauge only; the next ttns_tdvp_step returns
                                it to the root)                              */

typedef struct {
  double re, im;
} ttns_c64;

/* One operator-sum term: coef * op_a (at node_a) (x) op_b (at node_b).
 * node_b = -1 marks an on-site term.  Hermitian conjugate pairs are listed
 * explicitly by the caller (the sum must be Hermitian; ttns_build checks). */
typedef struct {
  int32_t node_a, op_a;
  int32_t node_b, op_b;
  double coef;
} ttns_term;

/* A tree, its Hamiltonian and its initial product state. */
typedef struct {
  int32_t n_nodes;
  const int32_t *parent;     /* n_nodes, pre-order (see conventions)        */
  const int32_t *phys_dim;   /* n_nodes, >= 1 (ER nodes: 1)                 */
  const int32_t *bond_dim;   /* n_nodes, requested D of edge (i, parent[i]);
                                clamped to what either side can carry       */
  int32_t n_ops;
  const int32_t *op_dim;     /* n_ops                                        */
  const ttns_c64 *op_data;   /* the n_ops matrices, concatenated             */
  int32_t n_terms;
  const ttns_term *terms;
  const ttns_c64 *init_local;/* phys_dim[i] amplitudes per node, in node order;
                                node i's tensor starts as an isometry whose
                                first column is init_local(i) (x) children's
                                first states, completed by unit vectors     */
  int32_t n_observe;         /* local operators recorded every step          */
  const int32_t *observe_node;
  const int32_t *observe_op;
} ttns_tree;

/* The star Hamiltonian of Eq. (2): an electronic system H_S coupled through
 * operators A_i to bosonic environments with power-law spectral densities
 * J_i(w) = 2 pi alpha_i wc_i (w/wc_i)^s_i theta(wc_i - w), each mapped to a
 * chain of `length` sites (orthogonal-polynomial chain mapping, closed form).
 * Built into a tree whose root carries H_S and whose chain sites carry
 * eps_n b^+b and t_n (b_n^+ b_{n+1} + h.c.); the root couples to site 0 by
 * A_i (x) c0_i (b_0 + b_0^+).  Head occupations <b_0^+ b_0> are recorded. */
typedef struct {
  int32_t n_levels;
  const ttns_c64 *h_el;      /* n_levels^2                                   */
  const ttns_c64 *init_el;   /* n_levels amplitudes; chains start in vacuum  */
  int32_t n_chains;
  const ttns_c64 *coupling;  /* n_chains * n_levels^2: A_i                   */
  const double *alpha, *wc, *s;
  const int32_t *length, *local_dim, *bond_dim;
  int32_t topology;          /* 0: chains hang off the root; 1: binary tree
                                of ER nodes between the root and the chains */
  int32_t er_bond_dim;       /* D on root-ER and ER-ER edges                 */
  const int32_t *obb_dim;    /* n_chains or NULL: optimised boson basis of
                                each chain (Methods, "Tensor Network
                                States": an expandable Fock basis behind a
                                basis of obb_dim states).  With obb_dim[i]
                                > 0 every site of chain i is a node without
                                physical leg whose first child holds the
                                local_dim Fock states behind a bond of
                                dimension obb_dim[i] (the basis tensor) and
                                whose second child is the next site; 0 keeps
                                the plain chain                             */
  int32_t potential;         /* 0: the operator sum is H; 1: it is H - T, T
                                the environments' kinetic energy (sum over
                                each chain's normal modes of (w/2) P^2, i.e.
                                (1/2) p^T M p over the site momenta p, M the
                                chain's tridiagonal matrix): the operator of
                                the effective potential of Eq. (4), whose
                                context takes a state by ttns_copy_state    */
} ttns_star_model;

typedef struct {
  int32_t precision;         /* TTNS_FP64 / TTNS_FP32 / TTNS_BF16X3          */
  int32_t krylov_dim;        /* Lanczos dimension m, 1..16 (default 12)      */
  double breakdown_tol;      /* stop Lanczos at beta_j <= tol*|x| (1e-12)    */
  double rank_tol;           /* QR completion below tol*|A|_F (1e-8)        */
  int32_t record_capacity;   /* records kept on the device (>= 1)            */
  int32_t executor;          /* TTNS_EXEC_*                                  */
  uint32_t flags;            /* TTNS_FLAG_* (0 by default)                   */
  int32_t coop_workgroups;   /* TTNS_EXEC_COOPERATIVE: workgroups on the one
                                XCD (0: 32; capped at what fits on an XCD) */
} ttns_opts;

typedef struct ttns_ctx ttns_ctx;

/* Fill opts with the defaults named above. */
void ttns_default_opts(ttns_opts *opts);

/* Chain mapping of one environment (Methods, "Tensor Network States", and
 * "Interface to TTNS": the orthogonal-polynomial chain transformation of
 * Chin et al. 2010 that the paper cites), closed form of the hard-cutoff
 * power-law density J(w) = 2 pi alpha wc (w/wc)^s theta(wc - w):
 *   c0 = coupling of the system to site 0 (the reaction coordinate of
 *        Eq. (2)), eps[0..L-1] = site energies, hop[0..L-2] = hoppings.
 * Host pointers owned by the caller (hop may be NULL for L = 1).
 * TTNS_EINVAL for L < 1, wc <= 0, s <= -1, alpha < 0 or a NULL output. */
int ttns_ohmic_chain(double alpha, double wc, double s, int32_t L, double *c0,
                     double *eps, double *hop);

/* Device bytes ttns_build (ttns_star_build) needs for these trees, all trees
 * run together.  The trees are validated as by the build; *bytes receives
 * the size (host pointer).  TTNS_EINVAL / TTNS_ENUMERIC as for the build. */
int ttns_workspace_size(const ttns_tree *trees, int32_t n_trees,
                        const ttns_opts *opts, size_t *bytes);
int ttns_star_workspace_size(const ttns_star_model *models, int32_t n_models,
                             const ttns_opts *opts, size_t *bytes);

/* Build the TTNS of every tree (section "TTNS for vibronic quantum dynamics":
 * one tensor per node, bond dimension D per edge; the star form of Eq. (2)
 * or, with ER nodes, the tree of Fig. 2): validate the topology and the
 * Hermiticity of the operator sum, lay out the workspace, upload the
 * operators, initialise the product state (electronic level(s) given,
 * environments in their vacuum: the zero-temperature start of Methods) with
 * every non-root node an isometry towards the root, and build every
 * environment towards the root.
 *   trees / models: host descriptions, copied during the call.
 *   dev_ws: device memory of ws_bytes >= the size query, 256-byte aligned,
 *           owned by the caller and used by the context until ttns_destroy
 *           (the library never allocates device memory).
 *   hip_stream: hipStream_t (NULL: the default stream) that orders all device
 *           work of the context.
 *   *out: the new context (NULL on failure).  Records t = 0.
 * Errors: TTNS_EINVAL (topology, dims, operators, non-Hermitian sum, bond
 * dimension above 64, options), TTNS_ENUMERIC (non-finite inputs),
 * TTNS_ENOMEM (workspace too small), TTNS_EDEVICE (a HIP call failed). */
int ttns_build(const ttns_tree *trees, int32_t n_trees, const ttns_opts *opts,
               void *dev_ws, size_t ws_bytes, void *hip_stream, ttns_ctx **out);
int ttns_star_build(const ttns_star_model *models, int32_t n_models,
                    const ttns_opts *opts, void *dev_ws, size_t ws_bytes,
                    void *hip_stream, ttns_ctx **out);

/* ttns_star_build without a caller workspace, for callers that cannot
 * allocate device memory (code that forbids hipMalloc, tight serving loops):
 * the context lives in a static device array of 64 MiB per device
 * (TTNS_ENOMEM if the trees need more; the size query tells), which every
 * device that loads the library holds until the process ends.  One live
 * context per device may use it: a second build on the same device fails
 * with TTNS_EINVAL until the first is destroyed.  Contexts built here run
 * their steps launch by launch on hip_stream (no graph is captured or
 * instantiated), so ttns_tdvp_step on them allocates nothing either and may
 * itself be captured by the caller.  The build, which uploads and
 * synchronises, must not be captured.  Calls on two such contexts cannot
 * overlap on one device (there is only one); TTNS_FLAG_AUTOTUNE is refused
 * (its timing events allocate). */
int ttns_star_build_noalloc(const ttns_star_model *models, int32_t n_models,
                            const ttns_opts *opts, void *hip_stream,
                            ttns_ctx **out);

/* The local effective Hamiltonian of one node, H_eff(t) of the section "TTNS
 * for vibronic quantum dynamics" (every tensor is evolved with an H_eff built
 * from the full many-body state; the same operator whose eigenvalues give the
 * energy surfaces of Eqs. (3)-(4) at the root).  First moves the
 * orthogonality centre of `tree` to `node` (QR + environment updates: a
 * gauge change only, the state is unchanged), then
 *   dev_out = H_eff(node) dev_in,
 * both device buffers of one node tensor (complex, node tensor layout,
 * shape of `node`), owned by the caller; they must not overlap.  The centre
 * stays at `node`; the next ttns_tdvp_step moves it back to the root.
 * Asynchronous on the context's stream.  TTNS_EINVAL for a bad tree / node
 * index or NULL buffers. */
int ttns_apply_heff(ttns_ctx *ctx, int32_t tree, int32_t node,
                    const void *dev_in, void *dev_out);

/* n_steps second-order time steps of size dt (inverse units of the
 * Hamiltonian's energies) of the time-dependent variational principle
 * (Methods, "Tensor Network States"; section "TTNS for vibronic quantum
 * dynamics": each tensor is evolved in turn with its H_eff) on every tree:
 * the pre-order sweep with h = dt/2 (node forward exp(-i h H_eff), then for
 * each child: QR towards it, environment update, bond matrix backward
 * exp(+i h H_bond), absorb) followed by the adjoint post-order sweep; the
 * local exponentials are Lanczos with krylov_dim vectors.  Observables are
 * recorded after every step.  Asynchronous: a numerical failure inside the
 * steps (TTNS_ENUMERIC) is reported by the next ttns_observe.
 * TTNS_EINVAL for n_steps < 0 or a non-finite dt. */
int ttns_tdvp_step(ttns_ctx *ctx, double dt, int32_t n_steps);

/* Copy an observable of `tree` to host memory (synchronises the stream):
 * the electronic populations and reduced density matrix of the root
 * (section "Fission dynamics in DP-Mes": populations of the diabatic states),
 * chain-head occupations, norm, energy, bond entanglement entropy (section
 * "TTNS for vibronic quantum dynamics": S = -Tr rho ln rho), the record
 * history, a node tensor, statistics.  `index` is the node for
 * TTNS_OBS_TENSOR / TTNS_OBS_ENTROPY.  host_out (caller-owned) holds n_out
 * doubles.  TTNS_EINVAL if n_out is too small or the kind / index is bad;
 * TTNS_ENUMERIC if a step of this tree produced a non-finite record or a QR
 * without completion vector (the values are then not returned, except for
 * TTNS_OBS_STATS, _RECORD_SIZE, _BOND_DIMS and _STEP_FLOPS). */
int ttns_observe(ttns_ctx *ctx, int32_t kind, int32_t tree, int32_t index,
                 double *host_out, size_t n_out);

/* Energy surfaces of the electronic system, Eqs. (3)-(4) (section "Fission
 * dynamics in DP-Mes"): with the orthogonality centre moved to the root
 * (a gauge change only), the bath states phi_i are the right singular
 * vectors of the root tensor matricised as electronic level x all bonds
 * (the system-environment Schmidt decomposition; retained while
 * s_i > rank_tol s_0, at most n of them), and the matrix
 *   M[(i n + j), (k n + l)] = <phi_i|<j| O |phi_k>|l>
 * of the context's operator sum O (H: Eq. (3), the total energy surfaces;
 * H - T for a model built with `potential`: Eq. (4), the potential energy
 * surfaces) is formed on the device from applications of the root's
 * effective operator.  host_values (cap doubles, cap >= n^2) receives the
 * eigenvalues of M in ascending order (r n of them), *n_bath the number r of
 * bath states, and host_matrix (optional, 2 (r n)^2 doubles: re, im,
 * row-major) M itself.  Synchronises the stream.  TTNS_EINVAL for bad
 * arguments or more than 8 electronic levels, TTNS_ENUMERIC for a zero
 * state. */
int ttns_energy_surfaces(ttns_ctx *ctx, int32_t tree, double rank_tol,
                         int32_t *n_bath, double *host_values,
                         double *host_matrix, size_t cap);

/* Give tree dst_tree of dst the state of tree src_tree of src (the same
 * topology and bond dimensions, possibly another operator sum, e.g. the
 * H - T of Eq. (4)): src's centre is moved to the root, every node tensor is
 * copied on the device, and dst rebuilds its environments towards the root
 * for its own operator sum.  Both contexts on the current device; src's
 * stream is synchronised first, dst's at the end.  dst's records are not
 * updated.  TTNS_EINVAL when the trees or any node shape differ. */
int ttns_copy_state(ttns_ctx *dst, int32_t dst_tree, ttns_ctx *src,
                    int32_t src_tree);

/* Kernels, for profiling.  Ids 0..15 are the one-operation kernels (their
 * device symbols are ttns::k_op<id>), 16..18 the matrix-core H_eff group
 * kernels ttns::k_mode<precision> for FP64, FP32 and BF16X3. */
#define TTNS_K_APPLY 0      /* scalar operator apply (environments, absorb)  */
#define TTNS_K_HEFF_LZ 1    /* scalar H_eff apply + Lanczos dots             */
#define TTNS_K_NORM 2
#define TTNS_K_SCALE 3
#define TTNS_K_ORTH1 4      /* Gram-Schmidt pass 1                           */
#define TTNS_K_ORTH2 5      /* Gram-Schmidt pass 2, next Krylov vector       */
#define TTNS_K_COMBINE 6    /* Krylov exponential and combination            */
#define TTNS_K_QR 7         /* guarded QR, one workgroup                     */
#define TTNS_K_CONTRACT 8   /* environment contraction                       */
#define TTNS_K_BOND 9       /* backward bond exponential                     */
#define TTNS_K_COPY 10
#define TTNS_K_DOT 11
#define TTNS_K_RECORD 12
#define TTNS_K_QR_WIDE 14   /* guarded QR, one phase over many workgroups    */
#define TTNS_K_MODE_FP64 16 /* matrix-core H_eff group                       */
#define TTNS_K_MODE_FP32 17
#define TTNS_K_MODE_BF16X3 18
#define TTNS_K_COUNT 19

/* With enable != 0, ttns_tdvp_step runs its kernels one by one (no graph)
 * with a pair of HIP events around every launch on the context's stream.
 * ttns_profile_read: average device time (ms) per launch, launches and
 * algorithmic flops per launch of the H_eff contraction (TTNS_K_HEFF_LZ and
 * TTNS_K_MODE_*) since the last reset.  ttns_profile_kernel: totals of one
 * kernel since the last reset (ms, launches, algorithmic flops, algorithmic
 * bytes: every operand read once and every result written once, 16 bytes per
 * complex entry). */
int ttns_profile(ttns_ctx *ctx, int32_t enable);
int ttns_profile_read(ttns_ctx *ctx, int32_t reset, double *avg_ms,
                      int64_t *launches, double *flops_per_launch);
int ttns_profile_kernel(ttns_ctx *ctx, int32_t kernel, double *total_ms,
                        int64_t *launches, double *flops, double *bytes);

/* Text report of the autotuner's measurements and choices (empty without
 * TTNS_FLAG_AUTOTUNE): one line per node class or QR shape.  Writes at most
 * n bytes including the terminating zero; *needed (optional) receives the
 * full length + 1. */
int ttns_tuning_report(const ttns_ctx* ctx, char* out, size_t n, size_t* needed);

/* Release the context (host memory, captured graphs, its capture stream);
 * the caller's workspace is not freed.  NULL is accepted. */
int ttns_destroy(ttns_ctx *ctx);

/* sizeof of the structs of this ABI as the library was compiled: out[0..n)
 * = ttns_c64, ttns_term, ttns_tree, ttns_star_model, ttns_opts, ttnn_config
 * (0 past the end), so that a binding can refuse a library built from other
 * headers.  TTNS_EINVAL for a NULL out or n < 1. */
int ttns_struct_sizes(size_t *out, int32_t n);

/* Message of the last failed call on `ctx`, or, with ctx = NULL, of the last
 * failed call of the calling thread (the only one for a build or size query
 * that produced no context).  The string stays valid until the next call
 * that fails on the same context / thread. */
const char *ttns_last_error(const ttns_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* TTNS_H */
