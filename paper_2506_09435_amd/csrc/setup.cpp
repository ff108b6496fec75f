// Host-side set-up: GLL data, horizontal geometry, mesh validation, column colouring.
//
// GLL nodes (nodal Lagrange P^p spectral elements, paper Sec. 3.1; GLL as the
// node family is the adopted reading): the interior nodes are the roots of
// P_p', found by Newton iteration with the second derivative taken from
// Legendre's differential equation (1-x^2) P'' = 2x P' - p(p+1) P.  Weights
// are 2 / (p(p+1) P_p(x_i)^2).  The derivative matrix uses barycentric
// weights lambda_j = 1 / prod_{m != j}(x_j - x_m):
//   D_ij = (lambda_j / lambda_i) / (x_i - x_j) (i != j), D_ii = -sum_{j != i} D_ij.
//
// Horizontal element coordinates follow the Gordon-Hall transfinite map of
// the element's four (straight or circular) edges; the horizontal Jacobian
// J_h is obtained by applying D to the nodal coordinates (isoparametric).

#include <algorithm>
#include <map>
#include <array>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "fnpf_internal.h"

namespace fnpf {

static void legendre_pair(int p, double x, double &pp, double &pm) {
  double a = 1.0, b = x;
  if (p == 0) {
    pp = 1.0;
    pm = 0.0;
    return;
  }
  for (int n = 1; n < p; ++n) {
    double c = ((2.0 * n + 1.0) * x * b - n * a) / (n + 1.0);
    a = b;
    b = c;
  }
  pp = b;
  pm = a;
}

// Nodal 1D filter matrix M = V diag(sigma) V^-1 (Sec. 3.2, modal filtering) with
// V[i][n] = Pt_n(x_i), Pt_n = sqrt((2n+1)/2) P_n, at the GLL nodes x_i.  V^-1 follows from the
// discrete orthogonality of the GLL rule: sum_i w_i Pt_n(x_i) Pt_m(x_i) = gamma_n delta_nm with
// gamma_n = 1 for n < p and gamma_p = (2p+1)/p (the rule integrates Pt_p^2 inexactly), so
// V^-1[n][i] = w_i Pt_n(x_i) / gamma_n.  sigma: the exponential filter, 1 up to the cutoff,
// exp(-alpha ((n - cutoff)/(p - cutoff))^order) above.
void modal_filter_matrix(int p, int cutoff, double alpha, int order, double *M) {
  const int n1 = p + 1;
  std::vector<double> x(n1), w(n1), D((size_t)n1 * n1), V((size_t)n1 * n1), sig(n1);
  gll_host(p, x.data(), w.data(), D.data());
  for (int i = 0; i < n1; ++i) {
    double pm = 1.0, pc = x[i];   // P_0, P_1
    for (int n = 0; n < n1; ++n) {
      double pn;
      if (n == 0) {
        pn = 1.0;
      } else if (n == 1) {
        pn = x[i];
      } else {
        pn = ((2.0 * n - 1.0) * x[i] * pc - (n - 1.0) * pm) / n;
        pm = pc;
        pc = pn;
      }
      V[(size_t)i * n1 + n] = std::sqrt((2.0 * n + 1.0) / 2.0) * pn;
    }
  }
  for (int n = 0; n < n1; ++n)
    sig[n] = n <= cutoff ? 1.0 : std::exp(-alpha * std::pow((double)(n - cutoff) / (p - cutoff), order));
  for (int i = 0; i < n1; ++i)
    for (int k = 0; k < n1; ++k) {
      double a = 0.0;
      for (int n = 0; n < n1; ++n) {
        const double gam = n < p ? 1.0 : (2.0 * p + 1.0) / p;
        a += V[(size_t)i * n1 + n] * sig[n] * w[k] * V[(size_t)k * n1 + n] / gam;
      }
      M[(size_t)i * n1 + k] = a;
    }
}

void gll_host(int p, double *x, double *w, double *D) {
  const int n1 = p + 1;
  std::vector<double> xs(n1);
  xs[0] = -1.0;
  xs[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double t = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, Pm;
      legendre_pair(p, t, P, Pm);
      double d1 = p * (Pm - t * P) / (1.0 - t * t);
      double d2 = (2.0 * t * d1 - p * (p + 1.0) * P) / (1.0 - t * t);
      double dt = d1 / d2;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    xs[i] = t;
  }
  std::sort(xs.begin(), xs.end());
  std::vector<double> lam(n1, 1.0);
  for (int j = 0; j < n1; ++j) {
    double prod = 1.0;
    for (int m = 0; m < n1; ++m)
      if (m != j) prod *= (xs[j] - xs[m]);
    lam[j] = 1.0 / prod;
  }
  for (int i = 0; i < n1; ++i) {
    if (x) x[i] = xs[i];
    if (w) {
      double P, Pm;
      legendre_pair(p, xs[i], P, Pm);
      w[i] = 2.0 / (p * (p + 1.0) * P * P);
    }
  }
  if (D) {
    for (int i = 0; i < n1; ++i) {
      double s = 0.0;
      for (int j = 0; j < n1; ++j) {
        if (i == j) continue;
        double v = (lam[j] / lam[i]) / (xs[i] - xs[j]);
        D[i * n1 + j] = v;
        s += v;
      }
      D[i * n1 + i] = -s;
    }
  }
}

namespace {

struct Pt {
  double x, y;
};

// point on an edge from a to b at reference parameter t in [-1, 1]
Pt edge_point(Pt a, Pt b, const double *arc, double t) {
  double s = 0.5 * (t + 1.0);
  if (arc == nullptr || arc[2] == 0.0) return {a.x + s * (b.x - a.x), a.y + s * (b.y - a.y)};
  double cx = arc[0], cy = arc[1], r = arc[2];
  double ta = std::atan2(a.y - cy, a.x - cx);
  double tb = std::atan2(b.y - cy, b.x - cx);
  double d = tb - ta;
  while (d > M_PI) d -= 2.0 * M_PI;
  while (d <= -M_PI) d += 2.0 * M_PI;
  double th = ta + d * s;
  return {cx + r * std::cos(th), cy + r * std::sin(th)};
}

}  // namespace

std::string build_host_mesh(const fnpf_mesh_desc &m, Ctx &c, std::vector<double> &hm, std::vector<uint8_t> &flags,
                            std::vector<int32_t> &cols, std::vector<double> &mlump_w, std::vector<double> &mlump_s) {
  char buf[256];
  const int dim = m.dim, p = m.p, n1 = p + 1;
  const int nh = dim == 3 ? n1 * n1 : n1;
  const int64_t n_eh = m.n_eh, n_s = m.n_s;
  c.dim = dim;
  c.p = p;
  c.nz = m.nz;
  c.n_eh = m.n_eh;
  c.n_s = n_s;
  c.nh = nh;
  c.np = nh * n1;
  c.ng = dim == 3 ? 6 : 3;
  c.n_v = n_s * (int64_t)(p * m.nz + 1);
  c.n_e = n_eh * m.nz;
  c.g = m.g;

  // node ids
  c.h_eh_nodes.assign(m.eh_nodes, m.eh_nodes + n_eh * nh);
  c.h_corner.assign(m.eh_corner, m.eh_corner + n_eh * (dim == 3 ? 8 : 2));
  if (m.eh_arc && dim == 3)
    c.h_arc.assign(m.eh_arc, m.eh_arc + n_eh * 12);
  else
    c.h_arc.clear();
  c.h_tags.assign((size_t)n_eh * 2 * (dim - 1), 0);
  if (m.eh_face_tag)
    for (size_t k = 0; k < c.h_tags.size(); ++k) c.h_tags[k] = m.eh_face_tag[k];
  std::vector<int32_t> count(n_s, 0);
  for (int64_t e = 0; e < n_eh; ++e) {
    for (int t = 0; t < nh; ++t) {
      int32_t id = m.eh_nodes[e * nh + t];
      if (id < 0 || id >= n_s) {
        std::snprintf(buf, sizeof buf, "eh_nodes[%lld][%d] = %d out of range [0, %lld)", (long long)e, t, id,
                      (long long)n_s);
        return buf;
      }
      for (int u = 0; u < t; ++u)
        if (m.eh_nodes[e * nh + u] == id) {
          std::snprintf(buf, sizeof buf, "element %lld repeats horizontal node %d", (long long)e, id);
          return buf;
        }
      count[id]++;
    }
  }
  for (int64_t n = 0; n < n_s; ++n)
    if (count[n] == 0) {
      std::snprintf(buf, sizeof buf, "horizontal node %lld is not used by any element", (long long)n);
      return buf;
    }

  // layer fractions and node-level sigma
  c.h_layer_s.resize(m.nz + 1);
  for (int l = 0; l <= m.nz; ++l) c.h_layer_s[l] = m.layer_s ? m.layer_s[l] : (double)l / m.nz;
  if (c.h_layer_s[0] != 0.0 || c.h_layer_s[m.nz] != 1.0) return "layer_s must start at 0 and end at 1";
  for (int l = 0; l < m.nz; ++l)
    if (!(c.h_layer_s[l + 1] > c.h_layer_s[l])) return "layer_s must be strictly increasing";
  std::vector<double> x(n1), w(n1), D(n1 * n1);
  gll_host(p, x.data(), w.data(), D.data());
  c.h_sigma.resize(p * m.nz + 1);
  for (int l = 0; l < m.nz; ++l)
    for (int k = 0; k <= p; ++k)
      c.h_sigma[l * p + k] = c.h_layer_s[l] + (c.h_layer_s[l + 1] - c.h_layer_s[l]) * 0.5 * (x[k] + 1.0);

  // horizontal coordinates at the element GLL nodes
  const int ncomp = dim == 3 ? kHm3 : kHm2;
  std::vector<double> xh(n_eh * nh * (dim - 1));
  for (int64_t e = 0; e < n_eh; ++e) {
    if (dim == 2) {
      double xa = m.eh_corner[e * 2 + 0], xb = m.eh_corner[e * 2 + 1];
      for (int i = 0; i < n1; ++i) xh[e * nh + i] = xa + (xb - xa) * 0.5 * (x[i] + 1.0);
      continue;
    }
    const double *cc = m.eh_corner + e * 8;
    Pt c0{cc[0], cc[1]}, c1{cc[2], cc[3]}, c2{cc[4], cc[5]}, c3{cc[6], cc[7]};
    const double *arc = m.eh_arc ? m.eh_arc + e * 12 : nullptr;
    for (int j = 0; j < n1; ++j) {
      for (int i = 0; i < n1; ++i) {
        double xi = x[i], et = x[j];
        Pt e0 = edge_point(c0, c1, arc ? arc + 0 : nullptr, xi);
        Pt e1 = edge_point(c1, c2, arc ? arc + 3 : nullptr, et);
        Pt e2 = edge_point(c3, c2, arc ? arc + 6 : nullptr, xi);
        Pt e3 = edge_point(c0, c3, arc ? arc + 9 : nullptr, et);
        double bx = 0.25 * ((1 - xi) * (1 - et) * c0.x + (1 + xi) * (1 - et) * c1.x + (1 + xi) * (1 + et) * c2.x +
                            (1 - xi) * (1 + et) * c3.x);
        double by = 0.25 * ((1 - xi) * (1 - et) * c0.y + (1 + xi) * (1 - et) * c1.y + (1 + xi) * (1 + et) * c2.y +
                            (1 - xi) * (1 + et) * c3.y);
        double px = 0.5 * (1 - et) * e0.x + 0.5 * (1 + et) * e2.x + 0.5 * (1 - xi) * e3.x + 0.5 * (1 + xi) * e1.x - bx;
        double py = 0.5 * (1 - et) * e0.y + 0.5 * (1 + et) * e2.y + 0.5 * (1 - xi) * e3.y + 0.5 * (1 + xi) * e1.y - by;
        int64_t o = (e * nh + j * n1 + i) * 2;
        xh[o] = px;
        xh[o + 1] = py;
      }
    }
  }
  // node coordinates (first image)
  c.h_node_xy.assign(n_s * (dim - 1), 0.0);
  {
    std::vector<char> seen(n_s, 0);
    for (int64_t e = 0; e < n_eh; ++e)
      for (int t = 0; t < nh; ++t) {
        int32_t id = m.eh_nodes[e * nh + t];
        if (seen[id]) continue;
        seen[id] = 1;
        for (int a = 0; a < dim - 1; ++a) c.h_node_xy[id * (dim - 1) + a] = xh[(e * nh + t) * (dim - 1) + a];
      }
  }
  c.h_xh = xh;
  // horizontal metrics and lumped masses
  hm.assign((size_t)ncomp * n_eh * nh, 0.0);
  mlump_w.assign(n_s, 0.0);
  mlump_s.assign(n_s, 0.0);
  const int64_t stride = n_eh * nh;
  for (int64_t e = 0; e < n_eh; ++e) {
    for (int t = 0; t < nh; ++t) {
      const int i = t % n1, j = t / n1;
      const int64_t o = e * nh + t;
      double det, ws;
      if (dim == 2) {
        double xx = 0.0;
        for (int mm = 0; mm < n1; ++mm) xx += D[i * n1 + mm] * xh[e * nh + mm];
        if (!(xx > 0.0)) {
          std::snprintf(buf, sizeof buf, "element %lld: non-positive horizontal Jacobian (corners reversed?)",
                        (long long)e);
          return buf;
        }
        hm[0 * stride + o] = 1.0 / xx;
        hm[1 * stride + o] = xx;
        det = xx;
        ws = w[i];
      } else {
        double xxi = 0, xet = 0, yxi = 0, yet = 0;
        for (int mm = 0; mm < n1; ++mm) {
          xxi += D[i * n1 + mm] * xh[(e * nh + j * n1 + mm) * 2];
          yxi += D[i * n1 + mm] * xh[(e * nh + j * n1 + mm) * 2 + 1];
          xet += D[j * n1 + mm] * xh[(e * nh + mm * n1 + i) * 2];
          yet += D[j * n1 + mm] * xh[(e * nh + mm * n1 + i) * 2 + 1];
        }
        det = xxi * yet - xet * yxi;
        if (!(det > 0.0)) {
          std::snprintf(buf, sizeof buf,
                        "element %lld: non-positive horizontal Jacobian at node %d (clockwise or tangled corners)",
                        (long long)e, t);
          return buf;
        }
        hm[0 * stride + o] = yet / det;    // (J_h^{-1})_00
        hm[1 * stride + o] = -xet / det;   // (J_h^{-1})_01
        hm[2 * stride + o] = -yxi / det;   // (J_h^{-1})_10
        hm[3 * stride + o] = xxi / det;    // (J_h^{-1})_11
        hm[4 * stride + o] = det;
        hm[5 * stride + o] = xxi;
        hm[6 * stride + o] = xet;
        hm[7 * stride + o] = yxi;
        hm[8 * stride + o] = yet;
        ws = w[i] * w[j];
      }
      int32_t id = m.eh_nodes[o];
      mlump_s[id] += ws * det;
      mlump_w[id] += ws * w[p] * det;
    }
  }

  // greedy colouring of columns: columns sharing a horizontal node get different colours
  std::vector<int64_t> off(n_s + 1, 0);
  for (int64_t n = 0; n < n_s; ++n) off[n + 1] = off[n] + count[n];
  std::vector<int32_t> adj(off[n_s]);
  {
    std::vector<int64_t> pos(off.begin(), off.end() - 1);
    for (int64_t e = 0; e < n_eh; ++e)
      for (int t = 0; t < nh; ++t) adj[pos[m.eh_nodes[e * nh + t]]++] = (int32_t)e;
  }
  std::vector<int32_t> colour(n_eh, -1);
  int ncol = 0;
  for (int64_t e = 0; e < n_eh; ++e) {
    uint64_t used = 0;
    for (int t = 0; t < nh; ++t) {
      int32_t id = m.eh_nodes[e * nh + t];
      for (int64_t q = off[id]; q < off[id + 1]; ++q) {
        int32_t o = adj[q];
        if (colour[o] >= 0) used |= (1ull << colour[o]);
      }
    }
    int cc = 0;
    while (cc < 64 && (used >> cc & 1ull)) ++cc;
    if (cc >= 64) return "column colouring needs more than 64 colours";
    colour[e] = cc;
    ncol = std::max(ncol, cc + 1);
  }
  c.colours.assign(ncol, ColourRange{0, 0});
  for (int64_t e = 0; e < n_eh; ++e) c.colours[colour[e]].count++;
  for (int k = 1; k < ncol; ++k) c.colours[k].offset = c.colours[k - 1].offset + c.colours[k - 1].count;
  cols.assign(n_eh, 0);
  {
    std::vector<int32_t> fill(ncol, 0);
    for (int64_t e = 0; e < n_eh; ++e) cols[c.colours[colour[e]].offset + fill[colour[e]]++] = (int32_t)e;
  }
  // first / last writer flags per (column, local node), in colour launch order
  flags.assign(n_eh * nh, 0);
  for (int64_t e = 0; e < n_eh; ++e) {
    for (int t = 0; t < nh; ++t) {
      int32_t id = m.eh_nodes[e * nh + t];
      int cmin = 1 << 30, cmax = -1;
      for (int64_t q = off[id]; q < off[id + 1]; ++q) {
        cmin = std::min(cmin, colour[adj[q]]);
        cmax = std::max(cmax, colour[adj[q]]);
      }
      uint8_t f = 0;
      if (colour[e] == cmin) f |= kFirst;
      if (colour[e] == cmax) f |= kLast;
      flags[e * nh + t] = f;
    }
  }
  // owner-computes assembly: every horizontal node belongs to the lowest-numbered column that
  // has it; a column's other nodes get face slots, numbered column by column in local order
  {
    std::vector<int32_t> owner(n_s, INT32_MAX);
    for (int64_t e = 0; e < n_eh; ++e)
      for (int t = 0; t < nh; ++t) {
        int32_t id = m.eh_nodes[e * nh + t];
        owner[id] = std::min(owner[id], (int32_t)e);
      }
    c.h_slot.assign(n_eh * nh, -1);
    int64_t ns = 0;
    for (int64_t e = 0; e < n_eh; ++e)
      for (int t = 0; t < nh; ++t) {
        int32_t id = m.eh_nodes[e * nh + t];
        if (owner[id] == e)
          flags[e * nh + t] |= kOwned;
        else
          c.h_slot[e * nh + t] = (int32_t)ns++;
        if (count[id] > 1) flags[e * nh + t] |= kShared;
      }
    if (ns >= INT32_MAX) return "too many face slots for the owner-computes apply";
    c.n_slots = ns;
    c.h_ps_node.clear();
    c.h_ps_slot.clear();
    c.h_ps_ptr.assign(1, 0);
    for (int64_t n = 0; n < n_s; ++n) {
      if (count[n] < 2) continue;
      c.h_ps_node.push_back((int32_t)n);
      for (int64_t q = off[n]; q < off[n + 1]; ++q) {
        const int32_t e = adj[q];   // increasing column id
        if (e == owner[n]) continue;
        for (int t = 0; t < nh; ++t)
          if (m.eh_nodes[(int64_t)e * nh + t] == n) {
            c.h_ps_slot.push_back(c.h_slot[(int64_t)e * nh + t]);
            break;
          }
      }
      c.h_ps_ptr.push_back((int32_t)c.h_ps_slot.size());
    }
    c.n_ps = (int)c.h_ps_node.size();

    // Tile assembly of the 3D owner-computes apply.  A tile is the tile_cols consecutive columns
    // of one workgroup; a node belongs to the tile of its owner column.  In each tile, the first
    // of the tile's columns that has a node is its representative: up to three other columns of
    // the tile pass their contributions through LDS exchange entries (at most tile_xmax per
    // tile), further ones get face slots of their own.  A representative stores y where its tile
    // owns the node and writes the tile's sum to a face slot elsewhere; the face pass adds the
    // slots of a node (in increasing slot order) to the owner's value.
    if (dim == 3) {
      const int tc = 256 / nh;
      c.tile_cols = tc;
      c.tile_xmax = tc * nh / 2;
      c.h_tslot.assign(n_eh * nh, -1);
      c.h_xch.assign(n_eh * nh * 4, (int16_t)-1);
      std::vector<std::vector<int32_t>> node_slots;        // per node with slots: its slots
      std::vector<int32_t> slot_of_node(n_s, -1);          // index into node_slots
      int64_t nts = 0;
      auto add_slot = [&](int32_t id) {
        if (slot_of_node[id] < 0) {
          slot_of_node[id] = (int32_t)node_slots.size();
          node_slots.emplace_back();
        }
        node_slots[slot_of_node[id]].push_back((int32_t)nts);
        return (int32_t)nts++;
      };
      std::vector<int64_t> rep(n_s, -1);                  // (column, local node) of the representative
      std::vector<int> nxr(n_s, 0);                        // exchange entries read by the representative
      for (int64_t t0 = 0; t0 < n_eh; t0 += tc) {
        const int64_t t1 = std::min<int64_t>(t0 + tc, n_eh);
        int xcount = 0;
        for (int64_t e = t0; e < t1; ++e)
          for (int t = 0; t < nh; ++t) {
            const int64_t o = e * nh + t;
            const int32_t id = m.eh_nodes[o];
            if (rep[id] < 0 || rep[id] / nh < t0) {        // first column of this tile with the node
              rep[id] = o;
              nxr[id] = 0;
              flags[o] |= kTRep;
              if (owner[id] / tc == t0 / tc)
                flags[o] |= kTOwn;
              else
                c.h_tslot[o] = add_slot(id);
              continue;
            }
            const int64_t r = rep[id];
            if (nxr[id] < 3 && xcount < c.tile_xmax) {
              c.h_xch[o * 4] = (int16_t)xcount;
              c.h_xch[r * 4 + 1 + nxr[id]] = (int16_t)xcount;
              ++nxr[id];
              ++xcount;
            } else {
              c.h_tslot[o] = add_slot(id);                // exchange full: a face slot of its own
            }
          }
      }
      if (nts >= INT32_MAX) return "too many face slots for the tile assembly";
      c.n_tslots = nts;
      c.h_tps_node.clear();
      c.h_tps_slot.clear();
      c.h_tps_ptr.assign(1, 0);
      for (int64_t n = 0; n < n_s; ++n) {
        if (slot_of_node[n] < 0) continue;
        c.h_tps_node.push_back((int32_t)n);
        for (int32_t sl : node_slots[slot_of_node[n]]) c.h_tps_slot.push_back(sl);
        c.h_tps_ptr.push_back((int32_t)c.h_tps_slot.size());
      }
      c.n_tps = (int)c.h_tps_node.size();
      // the owner tile's representative takes the dot product of nodes without face slots
      for (int64_t o = 0; o < n_eh * nh; ++o)
        if ((flags[o] & kTOwn) && slot_of_node[m.eh_nodes[o]] >= 0) flags[o] |= kTShared;
      // The geometry's face layout: the same contributions, placed by the position k of their
      // node in the list of nodes with slots, so that its face pass reads them in the order of
      // its threads: the owner tile's value at k, the node's first slot at n_tps + k, further
      // slots (in increasing slot order) from 2 n_tps on.
      {
        const int64_t ntp = c.n_tps;
        std::vector<int32_t> pos(nts, -1);
        c.h_gx_ptr.assign(1, 0);
        c.h_gx_slot.clear();
        for (int64_t k = 0; k < ntp; ++k) {
          const std::vector<int32_t> &sl = node_slots[slot_of_node[c.h_tps_node[k]]];
          pos[sl[0]] = (int32_t)(ntp + k);
          for (size_t q = 1; q < sl.size(); ++q) {
            pos[sl[q]] = (int32_t)(2 * ntp + (int64_t)c.h_gx_slot.size());
            c.h_gx_slot.push_back(pos[sl[q]]);
          }
          c.h_gx_ptr.push_back((int32_t)c.h_gx_slot.size());
        }
        std::vector<int32_t> kpos(n_s, -1);
        for (int64_t k = 0; k < ntp; ++k) kpos[c.h_tps_node[k]] = (int32_t)k;
        c.h_gslot.assign(n_eh * nh, -1);
        for (int64_t o = 0; o < n_eh * nh; ++o) {
          if (c.h_tslot[o] >= 0)
            c.h_gslot[o] = pos[c.h_tslot[o]];
          else if ((flags[o] & kTShared) != 0)
            c.h_gslot[o] = kpos[m.eh_nodes[o]];
        }
        c.n_gslots = 2 * ntp + (int64_t)c.h_gx_slot.size();
        if (c.n_gslots >= INT32_MAX) return "too many face slots for the tile assembly";
      }
    }
  }
  return "";
}


// Numbering of the same horizontal elements at degree pc < p (levels of the p-multigrid
// preconditioner).  It follows the topology of the fine numbering: a vertex is identified by its
// fine id, an edge node by the edge's two fine nodes next to its ends (their smaller id fixes a
// direction along the edge, so both elements of an edge agree) and its position, an interior
// node by its element.  Ids are column-blocked: each node belongs to the lowest-numbered column
// that has it; column by column, shared nodes first, then interior ones.
std::string coarse_numbering(const Ctx &f, int pc, std::vector<int32_t> &nodes, int64_t &n_s) {
  const int pf = f.p, n1f = pf + 1, n1c = pc + 1;
  const int dim = f.dim;
  const int nhf = dim == 3 ? n1f * n1f : n1f, nhc = dim == 3 ? n1c * n1c : n1c;
  if (pc < 1 || pc >= pf) return "coarse degree must lie in [1, p)";
  if (pc >= 2 && pf < 3) return "edge nodes of the coarse level need p >= 3";
  const int64_t n_eh = f.n_eh;
  auto fid = [&](int64_t e, int i, int j) -> int64_t { return f.h_eh_nodes[e * nhf + j * n1f + i]; };
  std::vector<std::array<int64_t, 3>> keys((size_t)n_eh * nhc);
  for (int64_t e = 0; e < n_eh; ++e) {
    for (int t = 0; t < nhc; ++t) {
      const int ic = t % n1c, jc = dim == 3 ? t / n1c : 0;
      const bool bi = ic == 0 || ic == pc, bj = dim == 2 || jc == 0 || jc == pc;
      std::array<int64_t, 3> k{};
      if (dim == 2) {
        k = bi ? std::array<int64_t, 3>{0, fid(e, ic == 0 ? 0 : pf, 0), 0} : std::array<int64_t, 3>{2, e, t};
      } else if (bi && bj) {
        k = {0, fid(e, ic == 0 ? 0 : pf, jc == 0 ? 0 : pf), 0};
      } else if (bi) {   // edge at xi = -1 or +1, position jc along eta
        const int i = ic == 0 ? 0 : pf;
        const int64_t a = fid(e, i, 1), b = fid(e, i, pf - 1);
        k = a < b ? std::array<int64_t, 3>{1, a, jc} : std::array<int64_t, 3>{1, b, pc - jc};
      } else if (bj) {   // edge at eta = -1 or +1, position ic along xi
        const int j = jc == 0 ? 0 : pf;
        const int64_t a = fid(e, 1, j), b = fid(e, pf - 1, j);
        k = a < b ? std::array<int64_t, 3>{1, a, ic} : std::array<int64_t, 3>{1, b, pc - ic};
      } else {
        k = {2, e, t};
      }
      keys[e * nhc + t] = k;
    }
  }
  std::map<std::array<int64_t, 3>, std::array<int64_t, 3>> info;   // key -> {count, owner, id}
  for (int64_t e = 0; e < n_eh; ++e)
    for (int t = 0; t < nhc; ++t) {
      auto it = info.find(keys[e * nhc + t]);
      if (it == info.end())
        info.emplace(keys[e * nhc + t], std::array<int64_t, 3>{1, e, -1});
      else
        it->second[0] += 1;
    }
  // shared nodes of every column (by owner column) first, then the interior ones, so that the
  // shared nodes of a node level are one contiguous range (coalesced face pass)
  int64_t next = 0;
  for (int pass = 0; pass < 2; ++pass)
    for (int64_t e = 0; e < n_eh; ++e)
      for (int t = 0; t < nhc; ++t) {
        auto &v = info[keys[e * nhc + t]];
        if (v[1] != e || v[2] >= 0) continue;
        if ((pass == 0) != (v[0] > 1)) continue;
        v[2] = next++;
      }
  n_s = next;
  nodes.resize((size_t)n_eh * nhc);
  for (size_t k = 0; k < nodes.size(); ++k) nodes[k] = (int32_t)info[keys[k]][2];
  return "";
}

// Degree-p Lagrange interpolation of a surface field at physical horizontal points (observation
// operators such as wave gauges).  An element contains a point when the Newton inverse of its
// isoparametric map, x(xi, eta) = sum_ij l_i(xi) l_j(eta) x_ij over its GLL node coordinates,
// lands in [-1, 1]^(dim-1) (to 1e-10); the first such element in element order is taken.  On an
// edge shared by two elements both give the same weights, since only the edge's nodes are nonzero.
namespace {
void lagrange_row(int p, const double *x, double t, double *L, double *dL) {
  for (int j = 0; j <= p; ++j) {
    double v = 1.0, d = 0.0;
    for (int m = 0; m <= p; ++m) {
      if (m == j) continue;
      const double f = (t - x[m]) / (x[j] - x[m]);
      d = d * f + v / (x[j] - x[m]);
      v *= f;
    }
    L[j] = v;
    if (dL) dL[j] = d;
  }
}
}  // namespace

std::string surface_interp_weights(const Ctx &c, int32_t n_pts, const double *pts, int32_t *node, double *wout) {
  const int p = c.p, n1 = p + 1, nh = c.nh, dm = c.dim - 1;
  std::vector<double> x(n1), wq(n1), D(n1 * n1), Li(n1), Lj(n1), dLi(n1), dLj(n1);
  gll_host(p, x.data(), wq.data(), D.data());
  char buf[160];
  for (int32_t k = 0; k < n_pts; ++k) {
    const double px = pts[k * dm], py = dm == 2 ? pts[k * dm + 1] : 0.0;
    bool found = false;
    for (int64_t e = 0; e < c.n_eh && !found; ++e) {
      const double *xe = c.h_xh.data() + e * nh * dm;
      double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
      for (int t = 0; t < nh; ++t)
        for (int a = 0; a < dm; ++a) {
          lo[a] = std::min(lo[a], xe[t * dm + a]);
          hi[a] = std::max(hi[a], xe[t * dm + a]);
        }
      // the element lies inside its node box up to its edge curvature: test a box widened by
      // a quarter of its size
      const double q[2] = {px, py};
      bool out = false;
      for (int a = 0; a < dm; ++a) {
        const double pad = 0.25 * (hi[a] - lo[a]) + 1e-12;
        if (q[a] < lo[a] - pad || q[a] > hi[a] + pad) out = true;
      }
      if (out) continue;
      double r[2] = {0.0, 0.0};
      bool conv = false;
      for (int it = 0; it < 60; ++it) {
        lagrange_row(p, x.data(), r[0], Li.data(), dLi.data());
        if (dm == 2) lagrange_row(p, x.data(), r[1], Lj.data(), dLj.data());
        double X[2] = {0, 0}, J[2][2] = {{0, 0}, {0, 0}};
        for (int t = 0; t < nh; ++t) {
          const int i = t % n1, j = t / n1;
          const double li = Li[i], lj = dm == 2 ? Lj[j] : 1.0;
          const double di = dLi[i], dj = dm == 2 ? dLj[j] : 0.0;
          for (int a = 0; a < dm; ++a) {
            const double v = xe[t * dm + a];
            X[a] += li * lj * v;
            J[a][0] += di * lj * v;
            if (dm == 2) J[a][1] += li * dj * v;
          }
        }
        double f0 = X[0] - q[0], f1 = dm == 2 ? X[1] - q[1] : 0.0, d0, d1;
        if (dm == 1) {
          d0 = f0 / J[0][0];
          d1 = 0.0;
        } else {
          const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
          d0 = (J[1][1] * f0 - J[0][1] * f1) / det;
          d1 = (-J[1][0] * f0 + J[0][0] * f1) / det;
        }
        r[0] -= d0;
        r[1] -= d1;
        if (!(std::fabs(r[0]) < 3.0 && std::fabs(r[1]) < 3.0)) break;   // diverging: not this element
        // reference coordinates are O(1); rounding of the physical residual (coordinates of
        // size |x| over a Jacobian of the element's half width) limits the last correction
        if (std::fabs(d0) + std::fabs(d1) < 1e-11) {
          conv = true;
          break;
        }
      }
      if (!conv || std::fabs(r[0]) > 1.0 + 1e-10 || std::fabs(r[1]) > 1.0 + 1e-10) continue;
      r[0] = std::min(1.0, std::max(-1.0, r[0]));
      r[1] = std::min(1.0, std::max(-1.0, r[1]));
      lagrange_row(p, x.data(), r[0], Li.data(), nullptr);
      if (dm == 2) lagrange_row(p, x.data(), r[1], Lj.data(), nullptr);
      for (int t = 0; t < nh; ++t) {
        node[(int64_t)k * nh + t] = c.h_eh_nodes[e * nh + t];
        wout[(int64_t)k * nh + t] = Li[t % n1] * (dm == 2 ? Lj[t / n1] : 1.0);
      }
      found = true;
    }
    if (!found) {
      std::snprintf(buf, sizeof buf, "point %d (%g, %g) lies outside the mesh", k, px, py);
      return buf;
    }
  }
  return "";
}

}  // namespace fnpf
