// Host-side geometry of the decomposition: node classes, subdomain interior
// boxes and their band orderings, and the unit-modulus element matrix K0.
//
// Section 1 of the paper splits Omega into non-overlapping subdomains whose
// common boundary is the skeleton Gamma; unknowns are then split into
// interior ones (each belonging to one subdomain) and interface ones
// (Section 2, eq. (NumberFour)).  On a structured grid cut along grid
// planes a node lies in more than one subdomain closure exactly when one of
// its coordinates is an internal cut, so:
//   interface  <=> some coordinate is an internal cut, and the node is free
//   interior   <=> otherwise, and not on a clamped face
// The interior nodes of a subdomain then form a box.  Each box is numbered
// with its longest axis slowest and its shortest axis fastest, which keeps
// the half bandwidth of K_{I_i I_i} at dim*(n_fast*n_mid + n_fast + 1) +
// dim - 1.  Each block is padded to a multiple of 64 rows with an identity
// block so that the batched kernels only ever see full 64-row blocks.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace edd {

// Unit-modulus element matrix by 2-point (per axis) Gauss quadrature on the
// unit element; exact for the bilinear/trilinear integrands.  2D is plane
// stress with unit thickness.  Strain order: xx, yy, (zz), then engineering
// shears xy, (yz, xz).
void element_matrix(int dim, double nu, double *K0) {
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  if (dim == 2) lam = 2.0 * mu * lam / (lam + 2.0 * mu);
  const int nc = dim == 2 ? 4 : 8;
  const int nd = dim * nc;
  const int ns = dim == 2 ? 3 : 6;
  double Dm[6][6] = {};
  for (int i = 0; i < dim; ++i) {
    for (int j = 0; j < dim; ++j) Dm[i][j] = lam;
    Dm[i][i] += 2.0 * mu;
  }
  for (int i = dim; i < ns; ++i) Dm[i][i] = mu;
  // corner offsets, counter-clockwise, z = 0 face first
  const int cx[8] = {0, 1, 1, 0, 0, 1, 1, 0};
  const int cy[8] = {0, 0, 1, 1, 0, 0, 1, 1};
  const int cz[8] = {0, 0, 0, 0, 1, 1, 1, 1};
  const double g0 = 0.5 - 0.5 / std::sqrt(3.0), g1 = 0.5 + 0.5 / std::sqrt(3.0);
  const double gp[2] = {g0, g1};
  for (int i = 0; i < nd * nd; ++i) K0[i] = 0.0;
  const int nq = dim == 2 ? 4 : 8;
  for (int qp = 0; qp < nq; ++qp) {
    const double xi[3] = {gp[qp & 1], gp[(qp >> 1) & 1], gp[(qp >> 2) & 1]};
    const double wq = dim == 2 ? 0.25 : 0.125;
    // shape-function gradients
    double G[8][3];
    for (int a = 0; a < nc; ++a) {
      const int o[3] = {cx[a], cy[a], cz[a]};
      for (int k = 0; k < dim; ++k) {
        double gk = o[k] ? 1.0 : -1.0;
        for (int m = 0; m < dim; ++m)
          if (m != k) gk *= o[m] ? xi[m] : 1.0 - xi[m];
        G[a][k] = gk;
      }
    }
    double B[6][24] = {};
    for (int a = 0; a < nc; ++a) {
      if (dim == 2) {
        B[0][2 * a] = G[a][0];
        B[1][2 * a + 1] = G[a][1];
        B[2][2 * a] = G[a][1];
        B[2][2 * a + 1] = G[a][0];
      } else {
        B[0][3 * a] = G[a][0];
        B[1][3 * a + 1] = G[a][1];
        B[2][3 * a + 2] = G[a][2];
        B[3][3 * a] = G[a][1];
        B[3][3 * a + 1] = G[a][0];
        B[4][3 * a + 1] = G[a][2];
        B[4][3 * a + 2] = G[a][1];
        B[5][3 * a] = G[a][2];
        B[5][3 * a + 2] = G[a][0];
      }
    }
    for (int i = 0; i < nd; ++i)
      for (int j = 0; j < nd; ++j) {
        double s = 0.0;
        for (int a = 0; a < ns; ++a)
          for (int b = 0; b < ns; ++b) s += B[a][i] * Dm[a][b] * B[b][j];
        K0[i * nd + j] += wq * s;
      }
  }
}

// Default theta for N subdomains: 0.5 at 4, +0.1 per factor 4, at most 0.75
// (the optimal values reported with Tables 1-3 for 4, 16, 64, 256).
double default_theta(int nsub) {
  if (nsub <= 4) return 0.5;
  const double t = 0.5 + 0.05 * std::log2((double)nsub / 4.0);
  return std::min(0.75, t);
}

int build_geometry(edd_problem *p, const edd_mesh_desc *d) {
  const int D = d->dim;
  p->g.dim = D;
  for (int a = 0; a < 3; ++a) {
    p->g.nel[a] = a < D ? d->nel[a] : 1;
    p->g.nn[a] = a < D ? d->nel[a] + 1 : 1;
  }
  p->clamp = d->clamp_faces;
  p->nu = d->nu;
  p->n_nodes = (int64_t)p->g.nn[0] * p->g.nn[1] * p->g.nn[2];
  p->n_el = (int64_t)p->g.nel[0] * p->g.nel[1] * (D == 3 ? p->g.nel[2] : 1);
  p->ndof = p->n_nodes * D;
  int nblk[3] = {1, 1, 1};
  for (int a = 0; a < D; ++a) {
    p->cuts[a].assign(d->cuts[a], d->cuts[a] + d->ncuts[a]);
    nblk[a] = d->ncuts[a] - 1;
  }
  for (int a = D; a < 3; ++a) p->cuts[a] = {0, 1};
  p->n_sub = nblk[0] * nblk[1] * nblk[2];

  // per-axis tables: internal-cut flag and block of non-cut coordinates
  std::vector<char> is_cut[3];
  for (int a = 0; a < 3; ++a) {
    const int nn = p->g.nn[a];
    is_cut[a].assign(nn, 0);
    if (a >= D) continue;
    for (size_t c = 1; c + 1 < p->cuts[a].size(); ++c) is_cut[a][p->cuts[a][c]] = 1;
  }
  auto clamped = [&](int a, int x) {
    if (a >= D) return false;
    if ((p->clamp >> (2 * a)) & 1) { if (x == 0) return true; }
    if ((p->clamp >> (2 * a + 1)) & 1) { if (x == p->g.nel[a]) return true; }
    return false;
  };

  // subdomain interior boxes; local axes shortest fastest, longest slowest
  struct Box {
    int lo[3], len[3], ax[3];  // len and ax by local axis
  };
  std::vector<Box> boxes(p->n_sub);
  for (int sz = 0; sz < nblk[2]; ++sz)
    for (int sy = 0; sy < nblk[1]; ++sy)
      for (int sx = 0; sx < nblk[0]; ++sx) {
        const int sid = sx + nblk[0] * (sy + nblk[1] * sz);
        const int b[3] = {sx, sy, sz};
        Box &bx = boxes[sid];
        int len[3];
        for (int a = 0; a < 3; ++a) {
          if (a >= D) { bx.lo[a] = 0; len[a] = 1; continue; }
          int lo = p->cuts[a][b[a]], hi = p->cuts[a][b[a] + 1];
          if (is_cut[a][lo] || clamped(a, lo)) ++lo;
          if (is_cut[a][hi] || clamped(a, hi)) --hi;
          bx.lo[a] = lo;
          len[a] = std::max(0, hi - lo + 1);
        }
        int ax[3] = {0, 1, 2};
        std::stable_sort(ax, ax + D, [&](int x, int y) { return len[x] < len[y]; });
        for (int a = 0; a < 3; ++a) {
          bx.ax[a] = ax[a];
          bx.len[a] = len[ax[a]];
        }
      }
  auto band_kd = [&](int l0, int l1, int n) {
    int kd = D == 2 ? D * (l0 + 1) + D - 1 : D * (l0 * l1 + l0 + 1) + D - 1;
    return std::max(0, std::min(kd, n - 1));
  };
  auto box_dofs = [&](const Box &bx) {
    return (int64_t)bx.len[0] * bx.len[1] * bx.len[2] * D;
  };

  // which interiors are dissected (3D only): the separator is the middle
  // plane across the slow axis; its dense block must fit one workgroup
  std::vector<double> work(p->n_sub);
  for (int i = 0; i < p->n_sub; ++i) {
    const int64_t n = box_dofs(boxes[i]);
    work[i] = (double)n * (band_kd(boxes[i].len[0], boxes[i].len[1], (int)n) + 1);
  }
  std::vector<double> sorted_work(work);
  std::sort(sorted_work.begin(), sorted_work.end());
  const double median = sorted_work.empty() ? 0.0 : sorted_work[sorted_work.size() / 2];
  std::vector<char> split(p->n_sub, 0);
  for (int i = 0; i < p->n_sub && D == 3 && p->dissect != 0; ++i) {
    const Box &bx = boxes[i];
    const int ns = D * bx.len[0] * bx.len[1];
    if (bx.len[2] < 5 || ns - 1 + 32 > 1024 || ns - 1 > 960) continue;
    const int64_t n = box_dofs(bx);
    // more band blocks than subdomains keeps more compute units streaming
    split[i] = p->dissect == 1 || work[i] > 1.5 * median ||
               (p->dissect == -1 && p->n_sub < p->n_cu && n >= 3000);
  }

  // band blocks, interior dofs subdomain by subdomain: [half a][half b][sep]
  p->subs.clear();
  p->seps.clear();
  int64_t dof_off = 0, fac_off = 0, w_off = 0, w_true = 0;
  auto add_block = [&](const Box &bx, int len2, int lo2, int dir, int kind, int sep,
                       bool dense) {
    SubDesc s{};
    for (int a = 0; a < 3; ++a) {
      s.ax[a] = bx.ax[a];
      s.len[a] = bx.len[a];
      s.lo[a] = bx.lo[a];
    }
    s.len[2] = len2;
    s.lo[bx.ax[2]] = lo2;
    s.dir = dir;
    s.kind = kind;
    s.sep = sep;
    s.n = (int)((int64_t)s.len[0] * s.len[1] * s.len[2] * D);
    s.kd = dense ? std::max(0, s.n - 1) : band_kd(s.len[0], s.len[1], s.n);
    s.np = std::max(64, (s.n + 63) / 64 * 64);
    s.dof_off = dof_off;
    s.fac_off = fac_off;
    dof_off += s.n;
    fac_off += (int64_t)s.np * (s.kd + 1);
    p->subs.push_back(s);
    return (int)p->subs.size() - 1;
  };
  for (int i = 0; i < p->n_sub; ++i) {
    const Box &bx = boxes[i];
    const int L = bx.len[2], lo2 = bx.lo[bx.ax[2]];
    if (!split[i]) {
      add_block(bx, L, lo2, 1, 0, -1, false);
      continue;
    }
    const int mid = L / 2;
    const int sid = (int)p->seps.size();
    SepDesc sd{};
    sd.a = add_block(bx, mid, lo2, 1, 1, sid, false);
    sd.b = add_block(bx, L - mid - 1, lo2 + L - 1, -1, 1, sid, false);
    sd.s = add_block(bx, 1, lo2 + mid, 1, 2, sid, true);
    sd.ns = p->subs[sd.s].n;
    sd.ldw = (sd.ns + 31) / 32 * 32;
    sd.w_off = w_off;
    w_off += 2 * (int64_t)sd.ns * sd.ldw;
    w_true += 2 * (int64_t)sd.ns * sd.ns;
    p->seps.push_back(sd);
  }
  p->n_blk = (int)p->subs.size();
  p->n_sep = (int)p->seps.size();
  p->w_entries = w_true;
  p->w_alloc = w_off;
  p->max_kd = 0;
  p->max_n = 0;
  p->max_np = 0;
  p->fac_entries_real = 0;
  for (const SubDesc &s : p->subs) {
    p->fac_entries_real += (int64_t)s.n * (s.kd + 1);
    p->max_kd = std::max(p->max_kd, s.kd);
    p->max_n = std::max(p->max_n, s.n);
    p->max_np = std::max(p->max_np, s.np);
  }
  p->n_idofs = dof_off;
  p->n_inodes = dof_off / D;
  p->fac_entries = fac_off;

  // node map, packed interior nodes, interface nodes
  std::vector<int> nmap(p->n_nodes, kDirichlet);
  p->inode.assign(p->n_inodes, -1);
  for (const SubDesc &s : p->subs) {
    const int64_t nodes = (int64_t)s.len[0] * s.len[1] * s.len[2];
    for (int64_t l = 0; l < nodes; ++l) {
      const int loc[3] = {(int)(l % s.len[0]), (int)((l / s.len[0]) % s.len[1]),
                          (int)(l / ((int64_t)s.len[0] * s.len[1]))};
      int x[3] = {0, 0, 0};
      for (int a = 0; a < 3; ++a)
        x[s.ax[a]] = s.lo[s.ax[a]] + (a == 2 ? s.dir : 1) * loc[a];
      const int64_t node = x[0] + (int64_t)p->g.nn[0] * (x[1] + (int64_t)p->g.nn[1] * x[2]);
      nmap[node] = (int)(s.dof_off + D * l);
      p->inode[s.dof_off / D + l] = (int)node;
    }
  }
  p->gnode.clear();
  for (int z = 0; z < p->g.nn[2]; ++z)
    for (int y = 0; y < p->g.nn[1]; ++y)
      for (int x = 0; x < p->g.nn[0]; ++x) {
        const int c[3] = {x, y, z};
        bool dir = false, cut = false;
        for (int a = 0; a < D; ++a) {
          dir = dir || clamped(a, c[a]);
          cut = cut || is_cut[a][c[a]];
        }
        const int64_t node = x + (int64_t)p->g.nn[0] * (y + (int64_t)p->g.nn[1] * z);
        if (dir) {
          nmap[node] = kDirichlet;
        } else if (cut) {
          nmap[node] = gamma_code((int)p->gnode.size());
          p->gnode.push_back((int)node);
        } else if (nmap[node] < 0) {
          return EDD_EINVAL;  // a free non-interface node outside every box
        }
      }
  p->n_gamma = (int64_t)p->gnode.size();

  // launch orders: most work first (round-robin dispatch over the XCDs then
  // spreads the large blocks); halves and whole interiors apart from
  // separators, which depend on them
  auto by_work = [&](int a, int b) {
    const SubDesc &x = p->subs[a], &y = p->subs[b];
    return (int64_t)x.n * (x.kd + 1) > (int64_t)y.n * (y.kd + 1);
  };
  p->order.resize(p->n_blk);
  std::iota(p->order.begin(), p->order.end(), 0);
  std::stable_sort(p->order.begin(), p->order.end(), by_work);
  p->order_leaf.clear();
  p->order_sep.clear();
  for (int b : p->order) (p->subs[b].kind == 2 ? p->order_sep : p->order_leaf).push_back(b);

  element_matrix(D, p->nu, p->K0);
  p->theta_default = default_theta(p->n_sub);

  // keep the node map for the upload
  p->nmap_host.swap(nmap);
  return EDD_OK;
}

}  // namespace edd
