// Internal declarations of the edd library (not part of the C ABI).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/edd.h"

namespace edd {

// Map value of a node (int32 per global node):
//   >= 0       packed interior dof of component 0
//   kDirichlet clamped node
//   <= -2      interface node, index = -(value) - 2
constexpr int kDirichlet = -1;

// correction network: layers and hidden width
constexpr int kCnnLayers = 4;
constexpr int kCnnWidth = 32;

// Directions of the flexible-CG window: stored in blocks of kWinBlock vectors,
// each allocated when the iteration first reaches it, at most kMaxWindow.
constexpr int kWinBlock = 256, kMaxWindow = 8192;
// row chunks of the window dots (their partial sums: kWinChunks * kMaxWindow)
constexpr int kWinChunks = 64;
// Scalar slots of p->scal_d (FP64 device scalars read back through the pinned
// p->scal_h): the interface solver below 528 and its window coefficients
// from 4096 on (api.hip), the preconditioner 528..1499 (kernels_pc.hip), the
// OC update 1536..1599 (topopt.hip), the network 1600..1605
// (kernels_cnn.hip), full GMRES 2048..4095 (gmres.hip).
constexpr int kScalTotal = 4096 + 2 * kMaxWindow;
// slots of the captured interface iteration (api.hip, kernels_vec.hip):
// iteration index k, first converged iteration + 1 (0: not yet), tol^2,
// r.r of the step, p.q of the step, r.r history (ring of kGHist)
constexpr int kSlotGK = 1700, kSlotGDone = 1701, kSlotGTol2 = 1702, kSlotGRR = 1703,
              kSlotGPQ = 1704, kSlotGHist = 1708, kGHist = 256;
__host__ __device__ inline int gamma_code(int g) { return -g - 2; }
__host__ __device__ inline int gamma_index(int code) { return -code - 2; }

// Geometry of the structured grid, passed to kernels by value.
struct Geom {
  int dim;
  int nn[3];   // nodes per axis (1 for unused axes)
  int nel[3];  // elements per axis (1 for unused axes)
};

// One subdomain's interior block K_{I_i I_i} in band storage.
// Interior nodes form the box lo[a] .. lo[a]+len[a]-1 (global node
// coordinates).  Local node index l = a + na*(b + nb*c) with (a, b, c) the
// coordinates along the axes ax[0] (fastest), ax[1], ax[2] (slowest);
// local dof p = dim*l + comp.  The lower Cholesky factor is stored by
// columns: entry (q, p), 0 <= q-p <= kd, at fac[fac_off + p*(kd+1) + q-p].
//
// A band block is a whole subdomain interior (kind 0) or, when the interior
// is dissected, one of its two halves (kind 1, ordered so that the plane next
// to the separator comes last: dir = -1 runs the slow axis downwards from
// lo) or the separator plane itself (kind 2, stored with full bandwidth).
struct SubDesc {
  int n;       // interior dofs
  int kd;      // half bandwidth
  int np;      // n rounded up to a multiple of 64; rows n..np-1 of the band
               // hold an identity block so every 64-row block is full
  int len[3];  // box length along local axes (fast, mid, slow)
  int ax[3];   // global axis of each local axis
  int lo[3];   // box origin, indexed by global axis
  int dir;     // +1, or -1: the slow local axis runs from lo downwards
  int kind;    // 0 whole interior, 1 half, 2 separator
  int sep;     // separator record of a dissected interior, else -1
  int64_t dof_off;  // offset in interior vectors
  int64_t fac_off;  // offset in band storage (entries)
};

// One subdomain's explicit local Schur complement S_i = K^i_GG -
// K^i_GI (K^i_II)^{-1} K^i_IG (its own elements only) on the m = dim*mg
// interface dofs of its closure, local order: the closure's interface nodes
// by node id, components fastest.  S_i is dense row-major at s_off; Y (the
// forward-substituted couplings, n x m row-major) at y_off; the apply's
// local output at l_off; the interface positions of the local nodes at
// g_off; the closure box (node coordinates c_lo, extents c_ext) maps to local
// interface node indices (or -1) at t_off; elements e_lo .. e_hi (inclusive).
struct SchurDesc {
  int blk;          // band block of the subdomain's interior
  int m, mg;
  int c_lo[3], c_ext[3];
  int e_lo[3], e_hi[3];
  int64_t s_off, y_off, l_off, g_off, t_off;
};

// what a captured preconditioner graph was recorded for
struct PcGraphKey {
  const double *r = nullptr;
  double *z = nullptr;
  int k = 0, inner = 0, weighting = 0;
  double theta = 0.0;
  int form = 0, mass = 0;
  bool operator==(const PcGraphKey &o) const {
    return r == o.r && z == o.z && k == o.k && inner == o.inner && weighting == o.weighting &&
           theta == o.theta && form == o.form && mass == o.mass;
  }
};

// A dissected interior: halves a, b and separator s (band block ids).  The
// last ns rows of each half couple to the ns separator dofs through
// W_h = L_h,tail^{-1} K(tail_h, S), stored row-major (tail row, separator
// column) at w_off (half a) and w_off + ns*ns (half b).
struct SepDesc {
  int a, b, s;
  int ns;
  int ldw;        // row stride of W_h: ns rounded up to 32, so that a row
                  // segment of a column strip starts on a 128-byte line
  int64_t w_off;  // W_a at w_off, W_b at w_off + ns * ldw
};

}  // namespace edd

// The handle.  Everything below lives in host memory except the *_d
// pointers, which are device allocations owned by the handle.
struct edd_problem {
  // geometry
  edd::Geom g{};
  int clamp = 0;
  double nu = 0.3;
  int ncuts[3] = {0, 0, 0};
  std::vector<int> cuts[3];
  int n_sub = 0;
  int64_t n_nodes = 0, ndof = 0, n_el = 0;
  int64_t n_gamma = 0, n_inodes = 0, n_idofs = 0;
  int factor_precision = EDD_F64;

  // host bookkeeping
  int dissect = -1;
  int n_cu = 256;          // compute units of the device
  int n_blk = 0;           // band blocks (subdomains, halves and separators)
  std::vector<edd::SubDesc> subs;   // band blocks
  std::vector<int> order;  // launch order of band blocks (largest first)
  std::vector<int> order_leaf, order_sep;  // halves and whole interiors / separators
  std::vector<edd::SepDesc> seps;
  int n_sep = 0;
  int64_t w_entries = 0;  // coupling entries, 2 ns^2 per separator
  int64_t w_alloc = 0;    // entries of the W buffers (rows padded to ldw)
  std::vector<int> inode, gnode, nmap_host;
  int64_t fac_entries = 0;
  int max_kd = 0, max_n = 0, max_np = 0;
  int64_t fac_entries_real = 0;  // band entries without the padding rows
  double K0[24 * 24];
  double theta_default = 0.5;

  // skeleton / preconditioner (host side)
  int64_t sk_nnz = 0;

  // device memory
  void *alloc_ctx = nullptr;
  void *(*alloc_fn)(void *, size_t) = nullptr;
  void (*free_fn)(void *, void *) = nullptr;
  std::vector<void *> allocations;
  hipStream_t stream = nullptr;
  int device = 0;
  size_t lds_limit = 65536;

  double *K0_d = nullptr;
  int *nmap_d = nullptr, *inode_d = nullptr, *gnode_d = nullptr;
  edd::SubDesc *subs_d = nullptr;
  int *order_d = nullptr;
  int *order_leaf_d = nullptr, *order_sep_d = nullptr;
  edd::SepDesc *seps_d = nullptr;
  // explicit local Schur complements (S apply by dense GEMVs), see SchurDesc
  int s_apply_mode = 0;       // 0: through the interior factors; 1: explicit S_i
  bool sc_ready = false;      // S_i formed for the current moduli
  int sc_max_m = 0, sc_max_mg = 0;
  std::vector<edd::SchurDesc> sc_desc;
  edd::SchurDesc *sc_desc_d = nullptr;
  int *sc_gl_d = nullptr, *sc_tab_d = nullptr, *sc_optr_d = nullptr, *sc_oent_d = nullptr;
  double *sc_S_d = nullptr, *sc_Y_d = nullptr, *sc_yl_d = nullptr;
  int64_t sc_S_len = 0, sc_Y_len = 0;
  double *W64_d = nullptr;  // separator couplings (see SepDesc)
  float *W32_d = nullptr;
  int *info_d = nullptr;     // per-subdomain factorisation status
  double *E_d = nullptr;     // element moduli (FP64 copy)
  double *fac64_d = nullptr;  // band storage (padded allocation)
  int64_t fac_padded = 0;
  float *fac32_d = nullptr;
  double *rac64_d = nullptr;  // row-major copies used by the backward sweep
  float *rac32_d = nullptr;
  bool have_moduli = false;
  int solve_variant[2] = {0, 0};  // substitution variant, FP64 / FP32 factors
  int apply_variant[3] = {0, 0, 0};  // node-tile shape of the element kernel (0..2) for
                                     // all nodes, interior targets, interface targets
  double *tune_y_d = nullptr;     // output buffer of the element-kernel timings

  // skeleton operators of the interface preconditioner
  int sk_state = -1;            // weighting the device operators hold (-1 none)
  int64_t sk_n = 0;             // skeleton elements (edges 2D / faces 3D)
  int sk_npe = 0;               // nodes per skeleton element
  int *sk_adj_d = nullptr;      // [sk_n][2] neighbouring volume elements
  double *sk_w_d = nullptr;     // [sk_n] element weights
  int *skL_rowptr_d = nullptr, *skL_col_d = nullptr;
  double *skL_val_d = nullptr;
  int *skC_ptr_d = nullptr;     // contributions of each L entry
  int *skC_elem_d = nullptr, *skC_ab_d = nullptr;
  int *skN_ptr_d = nullptr, *skN_elem_d = nullptr;  // skeleton elements per node
  double *skM_d = nullptr;      // lumped mass (diagonal)
  double *skMc_val_d = nullptr; // consistent mass, values in the pattern of L
  double *skMcdiag_d = nullptr; // its diagonal
  double sk_Me[16] = {};        // skeleton element mass matrix (unit element)
  double sk_cheb_lo = 0.0, sk_cheb_hi = 0.0;  // bounds of diag(M)^{-1} M
  double *skLdiag_d = nullptr;  // diagonal of L (current weighting)
  double *skL0diag_d = nullptr; // diagonal of the unweighted L
  double *skS_d = nullptr;      // face-block scaling sqrt(Ldiag / L0diag)
  double sk_Le[16] = {}, sk_rowsum = 0.0;
  int n_faces = 0, n_face_classes = 0, n_rest = 0, max_face_m = 0;
  int *face_ptr_d = nullptr;    // [n_faces+1] start of each face in face_node
  int *face_node_d = nullptr;   // gamma indices, node-id order inside a face
  int *face_class_d = nullptr;  // class of each face
  int *face_blk_d = nullptr;    // workgroup -> face (-1: none), see precond_setup
  int n_face_blocks = 0;
  int64_t *class_off_d = nullptr;  // offset of each class inverse
  int *rest_d = nullptr;        // gamma indices of cross-point nodes
  double *face_inv_d = nullptr; // dense inverses of the unweighted face blocks
  int64_t face_inv_entries = 0;
  // Lanczos / inner PCG work space
  int pc_kcap = 0;
  double *pc_Q_d = nullptr;     // basis vectors
  double *pc_v_d[9] = {};       // work vectors (gamma-sized)
  double *pc_MQ_d = nullptr;    // M times the basis vectors (consistent M)
  double *pc_h = nullptr;       // pinned host buffer for coefficients

  // captured interface iterations (use_graphs >= 2)
  hipGraphExec_t fcg_graph = nullptr;
  int64_t fcg_graph_key[12] = {};
  double *gr_p_d = nullptr, *gr_q_d = nullptr;  // new direction and its S product

  // captured preconditioner applies (device-resident form)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t pc_graph = nullptr;
  edd::PcGraphKey pc_graph_key;

  // work buffers
  double *w_I[3] = {nullptr, nullptr, nullptr};  // interior vectors
  double *w_G[8] = {};                           // gamma vectors
  double *w_full[2] = {nullptr, nullptr};        // full nodal vectors
  double *partials_d = nullptr;
  double *scal_d = nullptr;
  double *scal_h = nullptr;  // pinned
  size_t partials_len = 0;

  // flexible Krylov window (directions P and S P)
  std::vector<double *> winP_blk, winQ_blk;  // kWinBlock directions each
  // device copies of the block addresses: P blocks, then Q blocks from
  // kMaxWindow / kWinBlock on (host copy for the stream-ordered upload)
  double **win_tab_d = nullptr;
  double *win_tab_h[2 * edd::kMaxWindow / edd::kWinBlock] = {};

  // preconditioner scratch (Lanczos basis etc.)
  double *pc_d = nullptr;
  size_t pc_len = 0;
  // mixed-mode outer iteration vectors
  double *outer_d = nullptr;
  size_t outer_len = 0;

  // correction network (kernels_cnn.hip)
  int64_t cnn_nparams = 0;
  int64_t cnn_off[edd::kCnnLayers] = {};
  int cnn_t = 0;           // Adam steps taken
  int cnn_matrix_cores = 0;  // hidden layers' forward on the FP16 matrix cores
  double cnn_nfree = 0.0;  // free dofs (rms normalisation)
  float *cnn_master_d = nullptr, *cnn_m_d = nullptr, *cnn_v_d = nullptr,
        *cnn_grad_d = nullptr, *cnn_part_d = nullptr, *cnn_target_d = nullptr;
  __half *cnn_w16_d = nullptr;
  float *cnn_act_d[5] = {};  // features, three hidden activations, output
  float *cnn_g_d[2] = {};    // activation gradients (ping-pong)
  double *cnn_r_d = nullptr, *cnn_dir_d = nullptr;  // residual and proposal

  int last_hip_error = 0;

  // full-system GMRES (gmres.hip): Arnoldi basis V ((cap+1) x ndof),
  // preconditioned directions Z (cap x ndof), work vectors
  int gm_cap = 0;
  double *gm_V = nullptr, *gm_Z = nullptr, *gm_w = nullptr;
  double *gm_vG = nullptr, *gm_zG = nullptr, *gm_tI = nullptr;

  // topology optimisation work vectors (n_el each): element energies,
  // moduli, updated densities (topopt.hip)
  double *to_s_d = nullptr, *to_E_d = nullptr, *to_rho_d = nullptr;

  // address of the static work array of edd_apply_S_noalloc on this
  // handle's device (noalloc.hip)
  double *scratch_d = nullptr;

  // kernel timing (edd_set_kernel_timing)
  bool kt_enabled = false;
  struct Pending { int kind; hipEvent_t a, b; };
  std::vector<Pending> kt_pending;
  std::vector<hipEvent_t> kt_pool;
  int64_t kt_count[EDD_KT_COUNT] = {};
  double kt_ms[EDD_KT_COUNT] = {};
};

namespace edd {

// ---- launchers implemented in the .hip files ----------------------------
// kernels_fe.hip
void launch_apply_full(edd_problem *p, const double *u, double *y);
void launch_apply_mapped(edd_problem *p, const int *tgt, int64_t ntgt,
                         const double *xI, double sI, const double *xG,
                         double sG, const double *base_global, double sy,
                         double *out);
void launch_assemble_band(edd_problem *p);
void launch_gather(edd_problem *p, const int *nodes, int64_t n,
                   const double *full, double *packed);
// u = (uI, uG) as a full nodal vector, zero on clamped dofs; uI may be
// null (interior entries zero)
void launch_scatter_solution(edd_problem *p, const double *uI,
                             const double *uG, double *u);
void launch_check_moduli(edd_problem *p, const double *E, double *flag);
void launch_convert_moduli(edd_problem *p, const void *E, int dtype);
void launch_mask_dirichlet(edd_problem *p, double *v);

// kernels_factor.hip
void launch_band_cholesky(edd_problem *p);
void launch_band_layouts(edd_problem *p);

// kernels_band.hip
void launch_band_solve(edd_problem *p, int precision, const double *b,
                       double *x);
bool band_solve_variant_ok(const edd_problem *p, int v);

// schur.hip / kernels_fe.hip: explicit local Schur complements
int schur_setup(edd_problem *p);   // tables and storage; EDD_EINVAL if not eligible
int schur_form(edd_problem *p);    // S_i from the current moduli and FP64 factors
void schur_apply(edd_problem *p, const double *v, double *y);
void launch_schur_couplings(edd_problem *p);  // Y_i = K^i_IG (rows of the band order)
void launch_schur_kgg(edd_problem *p);        // S_i += K^i_GG
constexpr int kBandSolveVariants = 7;
constexpr int kApplyVariants = 3;  // node-tile shapes of the element kernel

// kernels_vec.hip
// dots: out[k] = sum_i a_k[i] * b_k[i] for k < nd (nd <= 4), written to
// p->scal_d[slot + k].  Deterministic two-stage reduction.
void launch_dots(edd_problem *p, int64_t n, int nd, const double *const *a,
                 const double *const *b, int slot);
// y = a*x + b*y
void launch_axpby(edd_problem *p, int64_t n, double a, const double *x,
                  double b, double *y);
void launch_copy(edd_problem *p, int64_t n, const double *x, double *y);
void launch_fill(edd_problem *p, int64_t n, double v, double *y);
void launch_fill_f32(edd_problem *p, int64_t n, float *y);
// x += alpha*pv; r -= alpha*q with alpha = scal[num]/scal[den]
// also writes r.r to scal[slot] and copies scal[den] to scal[copy_dst];
// a breakdown step (scal[den] <= 0, alpha not finite) changes nothing and
// sets scal[flag_slot] = 1
void launch_cg_update(edd_problem *p, int64_t n, int num, int den,
                      double *x, const double *pv, double *r,
                      const double *q, int slot, int copy_dst, int flag_slot);
void launch_reduce(edd_problem *p, int nblocks, int stride, int nout, int slot);
size_t band_solve_lds_bytes(const edd_problem *p, int precision);
// padding (entries) around band storage; see kernels_band.hip and
// kernels_factor.hip
constexpr int64_t kBandPadFront = 128;
int64_t band_pad_back(int max_kd);

// Raise a kernel's dynamic LDS limit to the device's, once per (kernel,
// device); thread-safe.
void set_lds_limit_once(const void *kernel, const edd_problem *p);

// Lane `lane`'s value, broadcast to the whole wavefront.
template <typename T>
__device__ inline T lane_bcast(T v, int lane);
template <>
__device__ inline double lane_bcast<double>(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <>
__device__ inline float lane_bcast<float>(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
void element_matrix(int dim, double nu, double *K0);
double default_theta(int nsub);
int build_geometry(edd_problem *p, const edd_mesh_desc *d);
// multi-dot against a window of m vectors (stride n): out[j] = <z, W_j>
void launch_window_dots(edd_problem *p, int64_t n, int m, const double *W,
                        const double *z, int slot);
// p = z - sum_j (scal[cslot+j] / scal[dslot+j]) P_j
void launch_window_combine(edd_problem *p, int64_t n, int m,
                           const double *P, int cslot, int dslot,
                           const double *z, double *pv);
// The same two steps with the window taken from the device iteration index
// k = scal[kSlotGK] (m = min(k, cap) newest directions of the ring, oldest
// first), so that they can run inside a captured graph: dots into
// scal[cbase + slot], and pv = z - sum (scal[cbase+slot]/scal[dbase+slot]) P_slot.
void launch_window_dots_dev(edd_problem *p, int64_t n, int cap, const double *W,
                            const double *z, int cbase);
void launch_window_combine_dev(edd_problem *p, int64_t n, int cap, const double *P,
                               int cbase, int dbase, const double *z, double *pv);
// The same two steps in the host-driven iteration, one launch each for the
// whole window: the m newest directions of a ring of capacity cap, oldest at
// slot first, slot s stored at tab[s / kWinBlock] + (s % kWinBlock) * n
// (tab a device array); dots into scal[cbase + slot].
void launch_ring_dots(edd_problem *p, int64_t n, int cap, int first, int m,
                      const double *const *tab, const double *z, int cbase);
void launch_ring_combine(edd_problem *p, int64_t n, int cap, int first, int m,
                         const double *const *tab, int cbase, int dbase, const double *z,
                         double *pv);
// ring[(k % cap) * n ...] = src
void launch_ring_store(edd_problem *p, int64_t n, int cap, const double *src, double *ring);
// end of a captured iteration: r.r into the history, p.q into
// scal[pqbase + k % cap], the convergence flag, k += 1
void launch_iter_end(edd_problem *p, int cap, int pqbase);
// full-vector residual norms over free dofs: scal[slot] = ||f - y||^2,
// scal[slot+1] = ||f||^2
void launch_residual_norms(edd_problem *p, const double *f, const double *y,
                           int slot);

// y = S v with t (n_idofs doubles) as the interior work vector (api.hip)
void apply_S_with(edd_problem *p, const double *v, double *y, int prec, double *t);
// S x = rhs by the interface flexible CG to a relative tolerance (api.hip)
int interface_solve(edd_problem *p, const double *rhs, double *x, double rel_tol,
                    const edd_solve_opts *o, edd_solve_stats *st, int maxit, int *iters);
// look up the static work array of edd_apply_S_noalloc (noalloc.hip)
int scratch_init(edd_problem *p);

// topology optimisation (topopt.hip)
int element_energies(edd_problem *p, const double *u, double *s);
int oc_update(edd_problem *p, const double *rho, const double *s, const edd_oc_params &o,
              double *rho_new, double *E_new, edd_oc_result *res);

// preconditioner (kernels_pc.hip)
int precond_apply(edd_problem *p, const double *r, double *z,
                  const edd_solve_opts *o, edd_solve_stats *st,
                  bool low_precision);
int precond_setup(edd_problem *p);
int skeleton_op(edd_problem *p, int which, int weighting, const double *x, double *y,
                double tol, int maxit);

// correction network (kernels_cnn.hip)
int cnn_setup(edd_problem *p, int width);
int cnn_set_params(edd_problem *p, const float *params);
int cnn_get_params(edd_problem *p, float *params);
// E: element moduli for the stiffness indicator (nullptr: the moduli set last)
int cnn_predict(edd_problem *p, const double *E, const double *r, double *d);
int cnn_loss_grad(edd_problem *p, const double *E, const double *r, const double *e,
                  float *grad, double *loss);
int cnn_train_step(edd_problem *p, const double *E, const double *r, const double *e,
                   double lr, double *loss);

// Records HIP events around the launches in its scope when timing is on.
struct KTimer {
  edd_problem *p;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  KTimer(edd_problem *p_, int kind_);
  ~KTimer();
};

// helpers (api.hip)
void *dev_alloc(edd_problem *p, size_t bytes);
int check_hip(edd_problem *p, hipError_t e);
int read_scalars(edd_problem *p, int first, int count);

}  // namespace edd
