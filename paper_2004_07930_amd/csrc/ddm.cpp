// ORAS set-up on the host: overlapping subdomains, Boolean partition of unity, local
// Robin operators (patterns + gather maps), nested-dissection ordering and the
// multifrontal symbolic analysis.  Numeric work (local values, LDL^T, coarse E) runs on
// the GPU (factor.hip, coarse.hip).
//
// Paper, section "Domain decomposition preconditioner", eq. (oras):
//   M1^{-1} = sum_i R_i^T D_i A_i^{-1} R_i
// Readings (the abstract leaves the construction to its references):
//  * overlap: delta layers, each adding every tet that shares a vertex with the set;
//  * D_i Boolean: a dof is owned by the lowest subdomain id whose own tets touch it, so
//    sum_i R_i^T D_i R_i = I and the prolongation is a pure gather;
//  * A_i: the tets of the overlapped subdomain, the physical boundary conditions, and the
//    first-order absorbing (Robin) term on every face whose neighbour tet is outside.
#include <cstdio>
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <numeric>
#include <set>
#include <thread>

#include "ddm.h"

namespace hz {

namespace {

int env_int(const char* name, int def) {
  const char* s = std::getenv(name);
  return s ? std::atoi(s) : def;
}

// ---------------------------------------------------------------- nested dissection

struct NDNode {
  std::vector<int32_t> piv;  // local dof ids
  int child[2] = {-1, -1};
  int nchild = 0;
};

struct NDContext {
  const Mesh* m;
  const std::vector<int64_t>* tets;  // local tet -> global tet
  const std::vector<int32_t>* ltd;   // local tet -> 20 local dofs
  std::vector<double> cen;           // local tet centroid (3)
  std::vector<double> vmin, vmax;    // per local tet, per axis, min/max vertex coordinate
  std::vector<uint32_t> stampL, stampR;
  uint32_t gen = 0;
  int leaf;
  std::vector<NDNode> nodes;
};

int nd_recurse(NDContext& c, std::vector<int32_t>& tets, std::vector<int32_t>& dofs) {
  auto make_leaf = [&]() {
    NDNode nd;
    nd.piv = dofs;
    std::sort(nd.piv.begin(), nd.piv.end());
    c.nodes.push_back(std::move(nd));
    return (int)c.nodes.size() - 1;
  };
  if ((int64_t)dofs.size() <= c.leaf || tets.size() < 2) return make_leaf();

  struct Split {
    std::vector<int32_t> EL, ER, sep, DL, DR;
  };
  auto evaluate = [&](const std::vector<int32_t>& EL, const std::vector<int32_t>& ER, Split& sp) {
    ++c.gen;
    const uint32_t g = c.gen;
    for (int32_t q : EL)
      for (int l = 0; l < 20; ++l) c.stampL[(*c.ltd)[q * 20 + l]] = g;
    for (int32_t q : ER)
      for (int l = 0; l < 20; ++l) c.stampR[(*c.ltd)[q * 20 + l]] = g;
    sp.sep.clear();
    sp.DL.clear();
    sp.DR.clear();
    for (int32_t d : dofs) {
      bool l = c.stampL[d] == g, r = c.stampR[d] == g;
      if (l && r)
        sp.sep.push_back(d);
      else if (l)
        sp.DL.push_back(d);
      else
        sp.DR.push_back(d);
    }
  };
  Split best;
  bool have = false;
  std::vector<double> xs;
  for (int ax = 0; ax < 3; ++ax) {
    xs.resize(tets.size());
    for (size_t i = 0; i < tets.size(); ++i) xs[i] = c.cen[3 * tets[i] + ax];
    std::vector<double> tmp = xs;
    std::nth_element(tmp.begin(), tmp.begin() + tmp.size() / 2, tmp.end());
    const double med = tmp[tmp.size() / 2];
    // snap the cut to the nearest vertex coordinate so that whole element layers stay together
    double x0 = med, bestd = INFINITY;
    for (int32_t q : tets)
      for (const double v : {c.vmin[3 * q + ax], c.vmax[3 * q + ax]}) {
        const double dd = std::fabs(v - med);
        if (dd < bestd) {
          bestd = dd;
          x0 = v;
        }
      }
    Split sp;
    for (size_t i = 0; i < tets.size(); ++i) (xs[i] < x0 ? sp.EL : sp.ER).push_back(tets[i]);
    if (sp.EL.empty() || sp.ER.empty()) continue;
    evaluate(sp.EL, sp.ER, sp);
    const size_t mn = std::min(sp.DL.size(), sp.DR.size());
    if (mn * 5 < dofs.size()) continue;  // too unbalanced
    if (!have || sp.sep.size() < best.sep.size()) {
      best = std::move(sp);
      have = true;
    }
  }
  if (!have) {  // fallback: split the tets at the median index along the widest axis
    int ax = 0;
    double wmax = -1;
    for (int a = 0; a < 3; ++a) {
      double lo = INFINITY, hi = -INFINITY;
      for (int32_t q : tets) {
        lo = std::min(lo, c.cen[3 * q + a]);
        hi = std::max(hi, c.cen[3 * q + a]);
      }
      if (hi - lo > wmax) {
        wmax = hi - lo;
        ax = a;
      }
    }
    std::vector<int32_t> s = tets;
    std::stable_sort(s.begin(), s.end(), [&](int32_t a, int32_t b) { return c.cen[3 * a + ax] < c.cen[3 * b + ax]; });
    best.EL.assign(s.begin(), s.begin() + s.size() / 2);
    best.ER.assign(s.begin() + s.size() / 2, s.end());
    evaluate(best.EL, best.ER, best);
  }
  if (best.sep.size() == dofs.size() || (best.DL.empty() && best.DR.empty())) return make_leaf();
  // restrict each side's tets to those touching its dofs
  auto restrict_tets = [&](std::vector<int32_t>& E, const std::vector<int32_t>& D) {
    ++c.gen;
    for (int32_t d : D) c.stampL[d] = c.gen;
    std::vector<int32_t> out;
    for (int32_t q : E) {
      bool hit = false;
      for (int l = 0; l < 20 && !hit; ++l) hit = c.stampL[(*c.ltd)[q * 20 + l]] == c.gen;
      if (hit) out.push_back(q);
    }
    E.swap(out);
  };
  restrict_tets(best.EL, best.DL);
  restrict_tets(best.ER, best.DR);
  NDNode nd;
  nd.piv = best.sep;
  std::sort(nd.piv.begin(), nd.piv.end());
  std::vector<int32_t> DL = std::move(best.DL), DR = std::move(best.DR), EL = std::move(best.EL),
                       ER = std::move(best.ER);
  tets.clear();
  tets.shrink_to_fit();
  dofs.clear();
  dofs.shrink_to_fit();
  int kids[2], nk = 0;
  if (!DL.empty()) kids[nk++] = nd_recurse(c, EL, DL);
  if (!DR.empty()) kids[nk++] = nd_recurse(c, ER, DR);
  nd.nchild = nk;
  for (int i = 0; i < nk; ++i) nd.child[i] = kids[i];
  c.nodes.push_back(std::move(nd));
  return (int)c.nodes.size() - 1;
}

// per-subdomain symbolic result
struct SubSym {
  std::vector<Front> fronts;           // local front ids = index; child/parent local
  std::vector<std::vector<int32_t>> U;  // update rows (positions)
};

void build_subdomain(const Mesh& m, const std::vector<int32_t>& part, const std::vector<int32_t>& owner,
                     const std::vector<int64_t>& v2t_ptr, const std::vector<int64_t>& v2t, int32_t i, int32_t delta,
                     std::vector<int32_t>& loc, std::vector<uint8_t>& inside, Subdomain& S, SubSym& sym, int leaf) {
  const int64_t T = m.T;
  // --- overlap: delta vertex-adjacency layers
  std::vector<int64_t> cur;
  // inside[t] = 1 + the tet's layer (0: outside): 1 for the non-overlapping part, k + 1 for
  // the tets the k-th growth step adds
  for (int64_t t = 0; t < T; ++t)
    if (part[t] == i) {
      cur.push_back(t);
      inside[t] = 1;
    }
  for (int32_t layer = 0; layer < delta; ++layer) {
    std::vector<int64_t> add;
    for (int64_t t : cur)
      for (int v = 0; v < 4; ++v) {
        const int64_t g = m.tets[4 * t + v];
        for (int64_t k = v2t_ptr[g]; k < v2t_ptr[g + 1]; ++k) {
          const int64_t u = v2t[k];
          if (!inside[u]) {
            inside[u] = (uint8_t)(layer + 2);
            add.push_back(u);
          }
        }
      }
    cur.insert(cur.end(), add.begin(), add.end());
  }
  std::sort(cur.begin(), cur.end());
  // --- local dofs R_i (sorted global ids)
  std::vector<int32_t> gd;
  gd.reserve(cur.size() * 4);
  for (int64_t t : cur)
    for (int l = 0; l < 20; ++l) gd.push_back(m.tet_dofs[t * 20 + l]);
  std::sort(gd.begin(), gd.end());
  gd.erase(std::unique(gd.begin(), gd.end()), gd.end());
  S.n = (int64_t)gd.size();
  for (int64_t k = 0; k < S.n; ++k) loc[gd[k]] = (int32_t)k;
  S.owned.resize(S.n);
  S.dir.resize(S.n);
  for (int64_t k = 0; k < S.n; ++k) {
    S.owned[k] = owner[gd[k]] == i;
    S.dir[k] = m.dirichlet[gd[k]];
  }
  S.layer.assign(S.n, (uint8_t)(delta + 1));
  for (int64_t t : cur)
    for (int l = 0; l < 20; ++l) {
      uint8_t& y = S.layer[loc[m.tet_dofs[t * 20 + l]]];
      y = std::min<uint8_t>(y, (uint8_t)(inside[t] - 1));
    }
  // --- Robin faces: physical impedance or a cut (neighbour outside the overlapped set)
  std::vector<uint8_t> robin(cur.size(), 0);
  for (size_t q = 0; q < cur.size(); ++q) {
    const int64_t t = cur[q];
    for (int f = 0; f < 4; ++f) {
      const int64_t nb = m.nbr[4 * t + f];
      const bool imp = m.tag[4 * t + f] == HZ_BC_IMPEDANCE;
      const bool cut = nb >= 0 && !inside[nb];
      if (imp || cut) robin[q] |= (uint8_t)(1u << f);
    }
  }
  build_pattern_and_incidence(m, cur, loc, S.n, S.rowptr, S.col, S.inc);
  S.tsel.assign(cur.begin(), cur.end());
  S.robin = std::move(robin);
  // --- nested dissection over the overlapped tets
  std::vector<int32_t> ltd(cur.size() * 20);
  for (size_t q = 0; q < cur.size(); ++q)
    for (int l = 0; l < 20; ++l) ltd[q * 20 + l] = loc[m.tet_dofs[cur[q] * 20 + l]];
  NDContext c;
  c.m = &m;
  c.tets = &cur;
  c.ltd = &ltd;
  c.leaf = leaf;
  c.cen.resize(cur.size() * 3);
  c.vmin.resize(cur.size() * 3);
  c.vmax.resize(cur.size() * 3);
  for (size_t q = 0; q < cur.size(); ++q)
    for (int d = 0; d < 3; ++d) {
      double s = 0, lo = INFINITY, hi = -INFINITY;
      for (int v = 0; v < 4; ++v) {
        const double x = m.coords[3 * (int64_t)m.tets[4 * cur[q] + v] + d];
        s += x;
        lo = std::min(lo, x);
        hi = std::max(hi, x);
      }
      c.cen[3 * q + d] = 0.25 * s;
      c.vmin[3 * q + d] = lo;
      c.vmax[3 * q + d] = hi;
    }
  c.stampL.assign(S.n, 0);
  c.stampR.assign(S.n, 0);
  std::vector<int32_t> all_t(cur.size()), all_d(S.n);
  std::iota(all_t.begin(), all_t.end(), 0);
  std::iota(all_d.begin(), all_d.end(), 0);
  const int root = nd_recurse(c, all_t, all_d);
  // post-order positions
  S.perm.clear();
  S.perm.reserve(S.n);
  S.ipos.assign(S.n, -1);
  std::vector<int> order;  // nodes in post-order
  {
    std::vector<std::pair<int, int>> st{{root, 0}};
    while (!st.empty()) {
      auto& [nd, k] = st.back();
      if (k < c.nodes[nd].nchild) {
        const int ch = c.nodes[nd].child[k++];
        st.push_back({ch, 0});
      } else {
        order.push_back(nd);
        st.pop_back();
      }
    }
  }
  std::vector<int> node2front(c.nodes.size(), -1);
  sym.fronts.clear();
  for (int nd : order) {
    Front F;
    F.pos0 = (int64_t)S.perm.size();
    F.p = (int64_t)c.nodes[nd].piv.size();
    for (int32_t d : c.nodes[nd].piv) {
      S.ipos[d] = (int32_t)S.perm.size();
      S.perm.push_back(d);
    }
    F.nchild = c.nodes[nd].nchild;
    for (int k = 0; k < F.nchild; ++k) F.child[k] = node2front[c.nodes[nd].child[k]];
    node2front[nd] = (int)sym.fronts.size();
    sym.fronts.push_back(F);
  }
  for (size_t fi = 0; fi < sym.fronts.size(); ++fi)
    for (int k = 0; k < sym.fronts[fi].nchild; ++k) sym.fronts[sym.fronts[fi].child[k]].parent = (int32_t)fi;
  // --- symbolic: update rows of every front (post-order, children first)
  sym.U.assign(sym.fronts.size(), {});
  std::vector<int64_t> mark(S.n, -1);
  for (size_t fi = 0; fi < sym.fronts.size(); ++fi) {
    Front& F = sym.fronts[fi];
    const int64_t end = F.pos0 + F.p;
    std::vector<int32_t> u;
    for (int64_t q = F.pos0; q < end; ++q) {
      const int32_t v = S.perm[q];
      for (int64_t k = S.rowptr[v]; k < S.rowptr[v + 1]; ++k) {
        const int32_t pc = S.ipos[S.col[k]];
        if (pc >= end && mark[pc] != (int64_t)fi) {
          mark[pc] = (int64_t)fi;
          u.push_back(pc);
        }
      }
    }
    for (int k = 0; k < F.nchild; ++k)
      for (int32_t pc : sym.U[F.child[k]])
        if (pc >= end && mark[pc] != (int64_t)fi) {
          mark[pc] = (int64_t)fi;
          u.push_back(pc);
        }
    std::sort(u.begin(), u.end());
    F.r = (int64_t)u.size();
    sym.U[fi] = std::move(u);
  }
  for (size_t fi = 0; fi < sym.fronts.size(); ++fi) {
    int lvl = 0;
    for (int k = 0; k < sym.fronts[fi].nchild; ++k) lvl = std::max(lvl, sym.fronts[sym.fronts[fi].child[k]].level + 1);
    sym.fronts[fi].level = lvl;
  }
  for (int64_t t : cur) inside[t] = 0;
  for (int64_t k = 0; k < S.n; ++k) loc[gd[k]] = -1;
  S.gdofs = std::move(gd);
}

// index of elimination position q inside front F (with update rows U); q must be one of
// the front's rows, anything else means the elimination tree is inconsistent
inline int64_t front_index(const Front& F, const std::vector<int32_t>& U, int64_t q) {
  if (q >= F.pos0 && q < F.pos0 + F.p) return q - F.pos0;
  auto it = std::lower_bound(U.begin(), U.end(), (int32_t)q);
  HZ_REQUIRE(it != U.end() && *it == q, HZ_ERR_STATE, "symbolic analysis: row missing from its front");
  return F.p + (it - U.begin());
}

}  // namespace

int64_t Ddm::device_bytes() const {
  int64_t b = 0;
  b += d_fronts.bytes() + d_urows.bytes() + d_emap.bytes() + d_gidx.bytes() + d_orig_src.bytes() +
       d_orig_dst.bytes() + d_own_src.bytes() + d_lrowptr.bytes() + d_lcol.bytes() + d_ldir.bytes() +
       d_lval.bytes() + d_level_fronts.bytes() + d_flf.bytes();
  b += d_factor.bytes + d_update.bytes + d_dinv.bytes;
  b += d_pou_ptr.bytes() + d_pou_pos.bytes() + d_pou_w.bytes();
  if (icc) b += (int64_t)icc->bytes();
  b += d_fwd_work.bytes() + d_bwd_work.bytes() + d_imap.bytes();
  for (int t = 0; t < 2; ++t) b += d_fwdm_work[t].bytes() + d_bwdm_work[t].bytes();
  if (coarse)
    b += coarse->d_zptr.bytes() + coarse->d_ztptr.bytes() + coarse->d_azptr.bytes() + coarse->d_zcol.bytes() +
         coarse->d_ztcol.bytes() + coarse->d_azcol.bytes() + coarse->d_zval.bytes() + coarse->d_ztval.bytes() +
         coarse->d_az.bytes() + coarse->d_az32.bytes() + coarse->d_E.bytes() + coarse->d_E32.bytes();
  return b;
}

void build_coarse_host(const Mesh& m, const hz_coarse_mesh* cm, CoarseSpace& cs);

std::shared_ptr<Ddm> build_ddm(Ctx* ctx, std::shared_ptr<Operator> op, const int32_t* partition, int32_t n_sub,
                               int32_t overlap, const hz_coarse_mesh* coarse, int precision, int pou,
                               int local_solver) {
  const double t0 = wall_time();
  const Mesh& m = *op->mesh;
  HZ_REQUIRE(partition && n_sub >= 1 && overlap >= 0, HZ_ERR_ARG, "hz_setup_ddm: bad arguments");
  HZ_REQUIRE(precision == HZ_PREC_C128 || precision == HZ_PREC_MIXED, HZ_ERR_ARG, "hz_setup_ddm: bad precision");
  HZ_REQUIRE(pou == HZ_POU_BOOLEAN || pou == HZ_POU_SMOOTH, HZ_ERR_ARG, "hz_setup_ddm: bad partition of unity");
  HZ_REQUIRE(local_solver == HZ_LOCAL_EXACT || local_solver == HZ_LOCAL_ICC || local_solver == HZ_LOCAL_ICC_A2,
             HZ_ERR_ARG,
             "hz_setup_ddm: bad local solver");
  HZ_REQUIRE(overlap <= 250, HZ_ERR_ARG, "hz_setup_ddm: overlap above 250 layers");
  std::vector<int32_t> part(partition, partition + m.T);
  std::vector<int64_t> cnt(n_sub, 0);
  for (int64_t t = 0; t < m.T; ++t) {
    HZ_REQUIRE(part[t] >= 0 && part[t] < n_sub, HZ_ERR_ARG, "hz_setup_ddm: partition id out of range");
    cnt[part[t]]++;
  }
  for (int32_t i = 0; i < n_sub; ++i) HZ_REQUIRE(cnt[i] > 0, HZ_ERR_ARG, "hz_setup_ddm: empty subdomain");
  auto d = std::make_shared<Ddm>();
  d->op = op;
  d->precision = precision;
  d->pou = pou;
  d->local_solver = local_solver;
  d->n_sub = n_sub;
  d->overlap = overlap;
  // owners: lowest subdomain whose own tets touch the dof
  std::vector<int32_t> owner(m.n, INT32_MAX);
  for (int64_t t = 0; t < m.T; ++t)
    for (int l = 0; l < 20; ++l) {
      int32_t& o = owner[m.tet_dofs[t * 20 + l]];
      o = std::min(o, part[t]);
    }
  // vertex -> tets
  std::vector<int64_t> v2t_ptr(m.V + 1, 0), v2t(m.T * 4);
  for (int64_t k = 0; k < m.T * 4; ++k) v2t_ptr[m.tets[k] + 1]++;
  for (int64_t v = 0; v < m.V; ++v) v2t_ptr[v + 1] += v2t_ptr[v];
  {
    std::vector<int64_t> fill(v2t_ptr.begin(), v2t_ptr.end() - 1);
    for (int64_t k = 0; k < m.T * 4; ++k) v2t[fill[m.tets[k]]++] = k / 4;
  }
  const int leaf = env_int("HZ_ND_LEAF", 256);
  d->subs.resize(n_sub);
  std::vector<SubSym> syms(n_sub);
  {
    const int nt = std::max(1, std::min<int>(n_sub, std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
    std::atomic<int32_t> next{0};
    std::vector<std::string> errs(nt);
    std::vector<std::thread> th;
    for (int w = 0; w < nt; ++w)
      th.emplace_back([&, w] {
        std::vector<int32_t> loc(m.n, -1);
        std::vector<uint8_t> inside(m.T, 0);
        try {
          for (int32_t i; (i = next.fetch_add(1)) < n_sub;)
            build_subdomain(m, part, owner, v2t_ptr, v2t, i, overlap, loc, inside, d->subs[i], syms[i], leaf);
        } catch (const std::exception& e) {
          errs[w] = e.what();
        }
      });
    for (auto& t : th) t.join();
    for (auto& e : errs) HZ_REQUIRE(e.empty(), HZ_ERR_STATE, "hz_setup_ddm: " + e);
  }
  auto phase = [&](const char* what) {
    if (ctx->trace) std::fprintf(stderr, "hz: setup %-34s %8.2f s\n", what, wall_time() - t0);
  };
  phase("subdomains, nested dissection, symbolic");
  // --- concatenate fronts, offsets
  int64_t vec = 0, csr = 0, rows = 0, Loff = 0, Uoff = 0, urow = 0, orig = 0;
  int max_level = 0;
  for (int32_t i = 0; i < n_sub; ++i) {
    Subdomain& S = d->subs[i];
    SubSym& sy = syms[i];
    S.vec_off = vec;
    S.csr_off = csr;
    S.row_off = rows;
    const int32_t base = (int32_t)d->fronts.size();
    for (size_t fi = 0; fi < sy.fronts.size(); ++fi) {
      Front F = sy.fronts[fi];
      F.sub = i;
      if (F.parent >= 0) F.parent += base;
      for (int k = 0; k < F.nchild; ++k) F.child[k] += base;
      F.L_off = Loff;
      Loff += F.ld() * F.p;
      F.U_off = Uoff;
      Uoff += F.r * F.r;
      F.rows_off = urow;
      F.emap_off = urow;
      urow += F.r;
      d->max_front = std::max(d->max_front, F.f());
      max_level = std::max(max_level, F.level);
      S.fronts.push_back((int32_t)d->fronts.size());
      d->fronts.push_back(F);
    }
    vec += S.n;
    csr += (int64_t)S.col.size();
    rows += S.n + 1;
  }
  d->n_local_total = vec;
  d->factor_entries = Loff;
  d->update_entries = Uoff;
  d->urows_total = urow;
  d->urows.resize(urow);
  d->emap.assign(urow, 0);
  // update rows, extend-add maps and original-entry scatter lists, one subdomain per task:
  // count each front's original entries, place them by a prefix sum (subdomain, then front
  // order), then fill every list at its offset
  auto each_sub = [&](const std::function<void(int32_t)>& body) {
    const int nt = std::max(1, std::min<int>(n_sub, std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
    std::atomic<int32_t> next{0};
    std::vector<std::string> errs(nt);
    std::vector<std::thread> th;
    for (int w = 0; w < nt; ++w)
      th.emplace_back([&, w] {
        try {
          for (int32_t i; (i = next.fetch_add(1)) < n_sub;) body(i);
        } catch (const std::exception& e) {
          errs[w] = e.what();
        }
      });
    for (auto& t : th) t.join();
    for (auto& e : errs) HZ_REQUIRE(e.empty(), HZ_ERR_STATE, "hz_setup_ddm: " + e);
  };
  each_sub([&](int32_t i) {
    const Subdomain& S = d->subs[i];
    for (size_t fi = 0; fi < S.fronts.size(); ++fi) {
      Front& F = d->fronts[S.fronts[fi]];
      int64_t cnt = 0;
      for (int64_t q = F.pos0; q < F.pos0 + F.p; ++q) {
        const int32_t v = S.perm[q];
        for (int64_t k = S.rowptr[v]; k < S.rowptr[v + 1]; ++k) cnt += S.ipos[S.col[k]] >= q;
      }
      F.orig_cnt = cnt;
    }
  });
  for (Front& F : d->fronts) {
    F.orig_off = orig;
    orig += F.orig_cnt;
  }
  d->orig_src.resize(orig);
  d->orig_dst.resize(orig);
  each_sub([&](int32_t i) {
    const Subdomain& S = d->subs[i];
    const SubSym& sy = syms[i];
    for (size_t fi = 0; fi < sy.fronts.size(); ++fi) {
      const Front& F = d->fronts[S.fronts[fi]];
      std::copy(sy.U[fi].begin(), sy.U[fi].end(), d->urows.begin() + F.rows_off);
      if (F.parent >= 0) {
        const Front& P = d->fronts[F.parent];
        const auto& UP = sy.U[(size_t)(F.parent - S.fronts[0])];
        for (int64_t k = 0; k < F.r; ++k) d->emap[F.emap_off + k] = (int32_t)front_index(P, UP, sy.U[fi][k]);
      }
      const int64_t ld = F.ld();
      int64_t o = F.orig_off;
      for (int64_t q = F.pos0; q < F.pos0 + F.p; ++q) {
        const int32_t v = S.perm[q];
        for (int64_t k = S.rowptr[v]; k < S.rowptr[v + 1]; ++k) {
          const int64_t pc = S.ipos[S.col[k]];
          if (pc < q) continue;
          d->orig_src[o] = S.csr_off + k;
          d->orig_dst[o] = (q - F.pos0) * ld + front_index(F, sy.U[fi], pc);
          ++o;
        }
      }
    }
  });
  d->orig_total = orig;
  phase("  update rows, scatter lists");
  // levels
  d->levels.assign(max_level + 1, Level{});
  for (size_t fi = 0; fi < d->fronts.size(); ++fi) d->levels[d->fronts[fi].level].fronts.push_back((int32_t)fi);
  std::vector<int32_t> lf;
  for (auto& L : d->levels) {
    std::stable_sort(L.fronts.begin(), L.fronts.end(),
                     [&](int32_t a, int32_t b) { return d->fronts[a].p > d->fronts[b].p; });
    for (int32_t fi : L.fronts) {
      const Front& F = d->fronts[fi];
      L.max_p = std::max(L.max_p, F.p);
      L.max_f = std::max(L.max_f, F.f());
      L.max_r = std::max(L.max_r, F.r);
      L.useful += F.p * (F.p + 1) / 2 + F.r * F.p;
      L.sum_f += F.f();
      L.sum_p += F.p;
    }
    d->level_off.push_back((int64_t)lf.size());
    lf.insert(lf.end(), L.fronts.begin(), L.fronts.end());
  }
  d->level_off.push_back((int64_t)lf.size());
  // Update (Schur) blocks live from their front's level until their parent's level has
  // absorbed them.  Place them in one arena with a best-fit allocator over those lifetimes: at
  // each level the new blocks are placed (largest p first) while the children being absorbed at
  // that level are still held, and only then are those children released.  The subdomains are
  // factored in groups of consecutive ids, one group after the other, each group packed from
  // offset 0: the arena then holds one group's blocks at a time.  A front's arithmetic does not
  // depend on the fronts it shares a launch with, so the grouping changes memory, not results.
  auto pack_arena = [&](const std::vector<std::vector<int32_t>>& lvl_fronts) -> int64_t {
    std::map<int64_t, int64_t> holes;          // offset -> length
    std::set<std::pair<int64_t, int64_t>> by_len;  // (length, offset) of the same holes
    int64_t arena = 0;
    auto drop = [&](std::map<int64_t, int64_t>::iterator it) {
      by_len.erase({it->second, it->first});
      return holes.erase(it);
    };
    auto take = [&](int64_t len) {
      auto b = by_len.lower_bound({len, INT64_MIN});
      if (b != by_len.end()) {  // the smallest hole that holds len (lowest offset among equals)
        const int64_t off = b->second, rest = b->first - len;
        drop(holes.find(off));
        if (rest > 0) {
          holes[off + len] = rest;
          by_len.insert({rest, off + len});
        }
        return off;
      }
      const int64_t off = arena;
      arena += len;
      return off;
    };
    auto give = [&](int64_t off, int64_t len) {
      auto nx = holes.lower_bound(off);
      if (nx != holes.begin()) {  // merge with the hole ending at off
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
          off = pv->first;
          len += pv->second;
          drop(pv);
        }
      }
      if (nx != holes.end() && off + len == nx->first) {  // and with the one starting at its end
        len += nx->second;
        drop(nx);
      }
      if (off + len == arena) {  // trailing hole: shrink the arena
        arena = off;
        return;
      }
      holes[off] = len;
      by_len.insert({len, off});
    };
    int64_t peak = 0;
    for (const auto& fl : lvl_fronts) {
      for (int32_t fi : fl) {
        Front& F = d->fronts[fi];
        F.U_off = F.r > 0 ? take(F.r * F.r) : 0;
        peak = std::max(peak, arena);
      }
      for (int32_t fi : fl) {
        const Front& F = d->fronts[fi];
        for (int k = 0; k < F.nchild; ++k) {
          const Front& C = d->fronts[F.child[k]];
          if (C.r > 0) give(C.U_off, C.r * C.r);
        }
      }
    }
    return peak;
  };
  {
    // group count: the smallest power of two whose arena fits next to the factor and the
    // local operators in the free device memory (HZ_FACTOR_GROUPS overrides)
    const int64_t elem = precision == HZ_PREC_MIXED ? (int64_t)sizeof(c64) : (int64_t)sizeof(c128);
    size_t fr = 0, tot = 0;
    HIP_CHECK(hipMemGetInfo(&fr, &tot));
    const double fixed = (double)d->factor_entries * elem + (double)csr * sizeof(c128) +
                         (double)d->orig_total * 16.0 + (double)vec * (elem + 16.0);
    const double budget = 0.85 * (double)fr - fixed;
    const int forced = env_int("HZ_FACTOR_GROUPS", 0);
    int G = forced > 0 ? std::min<int>(forced, n_sub) : 1;
    for (;;) {
      int64_t peak = 0;
      d->fgroup_off.clear();
      for (int g = 0; g <= G; ++g) d->fgroup_off.push_back((int32_t)((int64_t)n_sub * g / G));
      // each group's fronts per level, in the level's order (p descending)
      std::vector<int32_t> gsub(n_sub);
      for (int g = 0; g < G; ++g)
        for (int32_t i = d->fgroup_off[g]; i < d->fgroup_off[g + 1]; ++i) gsub[i] = g;
      std::vector<std::vector<std::vector<int32_t>>> gl(G, std::vector<std::vector<int32_t>>(d->levels.size()));
      for (size_t lv = 0; lv < d->levels.size(); ++lv)
        for (int32_t fi : d->levels[lv].fronts) gl[gsub[d->fronts[fi].sub]][lv].push_back(fi);
      for (int g = 0; g < G; ++g) peak = std::max(peak, pack_arena(gl[g]));
      d->update_entries = peak;
      if (forced > 0 || G >= n_sub || (double)peak * elem <= budget) break;
      G = std::min<int>(2 * G, n_sub);
    }
    // factor launches: the fronts of each (group, level), p descending
    d->flf.clear();
    d->flf_off.clear();
    for (int g = 0; g < G; ++g)
      for (const Level& L : d->levels) {
        d->flf_off.push_back((int64_t)d->flf.size());
        for (int32_t fi : L.fronts)
          if (d->fronts[fi].sub >= d->fgroup_off[g] && d->fronts[fi].sub < d->fgroup_off[g + 1]) d->flf.push_back(fi);
      }
    d->flf_off.push_back((int64_t)d->flf.size());
  }
  phase("fronts, levels, arena");
  if (ctx->trace)
    std::fprintf(stderr, "hz: setup factor %lld entries, arena %lld entries in %zu groups, %zu fronts, %zu levels\n",
                 (long long)d->factor_entries, (long long)d->update_entries, d->fgroup_off.size() - 1,
                 d->fronts.size(), d->levels.size());
  // local vector <-> global maps
  d->gidx.resize(vec);
  d->own_src.assign(m.n, -1);
  for (int32_t i = 0; i < n_sub; ++i) {
    const Subdomain& S = d->subs[i];
    for (int64_t q = 0; q < S.n; ++q) {
      const int32_t l = S.perm[q];
      d->gidx[S.vec_off + q] = S.gdofs[l];
      if (S.owned[l]) d->own_src[S.gdofs[l]] = S.vec_off + q;
    }
  }
  for (int64_t g = 0; g < m.n; ++g) HZ_REQUIRE(d->own_src[g] >= 0, HZ_ERR_STATE, "hz_setup_ddm: unowned dof");
  if (pou == HZ_POU_SMOOTH) {
    // raw weight 1 - layer / (overlap + 1), normalised over the subdomains holding the dof
    // (sums in subdomain order); per global dof its (position, weight) pairs in that order
    std::vector<double> tot(m.n, 0.0);
    std::vector<int64_t> cnt(m.n + 1, 0);
    for (int32_t i = 0; i < n_sub; ++i) {
      const Subdomain& S = d->subs[i];
      for (int64_t l = 0; l < S.n; ++l) {
        tot[S.gdofs[l]] += 1.0 - (double)S.layer[l] / (overlap + 1.0);
        cnt[S.gdofs[l] + 1]++;
      }
    }
    for (int64_t g = 0; g < m.n; ++g) cnt[g + 1] += cnt[g];
    std::vector<int64_t> pos(cnt[m.n]), fill(cnt.begin(), cnt.end() - 1);
    std::vector<double> wt(cnt[m.n]);
    for (int32_t i = 0; i < n_sub; ++i) {
      Subdomain& S = d->subs[i];
      S.pouw.resize(S.n);
      for (int64_t l = 0; l < S.n; ++l) {
        const int32_t g = S.gdofs[l];
        S.pouw[l] = (1.0 - (double)S.layer[l] / (overlap + 1.0)) / tot[g];
        const int64_t k = fill[g]++;
        pos[k] = S.vec_off + S.ipos[l];
        wt[k] = S.pouw[l];
      }
    }
    d->d_pou_ptr.upload(ctx, cnt);
    d->d_pou_pos.upload(ctx, pos);
    d->d_pou_w.upload(ctx, wt);
  }
  phase("  local-global maps");
  // --- device: front descriptors, maps, local operators
  std::vector<FrontDesc> fd(d->fronts.size());
  int64_t wrows = 0;
  std::vector<int32_t> imap;  // per front: 2 x f inverse extend-add maps (parent row -> child row, or -1)
  for (size_t fi = 0; fi < d->fronts.size(); ++fi) {
    const Front& F = d->fronts[fi];
    FrontDesc& x = fd[fi];
    x.L_off = F.L_off;
    x.U_off = F.U_off;
    x.rows_off = F.rows_off;
    x.emap_off = F.emap_off;
    x.orig_off = F.orig_off;
    x.orig_cnt = F.orig_cnt;
    x.vec_off = d->subs[F.sub].vec_off;
    x.w_off = wrows;
    wrows += F.f();
    x.imap_off = (int64_t)imap.size();
    imap.resize(imap.size() + 2 * F.f(), -1);
    for (int k = 0; k < F.nchild; ++k) {
      const Front& Cf = d->fronts[F.child[k]];
      for (int64_t q = 0; q < Cf.r; ++q) {
        const int32_t tgt = d->emap[Cf.emap_off + q];
        HZ_REQUIRE(tgt >= 0 && tgt < F.f(), HZ_ERR_STATE, "symbolic analysis: extend-add target out of range");
        imap[x.imap_off + k * F.f() + tgt] = (int32_t)q;
      }
    }
    d->factor_useful += F.p * (F.p + 1) / 2 + F.r * F.p;
    x.p = (int32_t)F.p;
    x.r = (int32_t)F.r;
    x.parent = F.parent;
    x.child0 = F.child[0];
    x.child1 = F.child[1];
    x.pos0 = (int32_t)F.pos0;
    x.ld = (int32_t)F.ld();
  }
  d->d_fronts.upload(ctx, fd);
  d->d_urows.upload(ctx, d->urows);
  d->d_emap.upload(ctx, d->emap);
  d->d_gidx.upload(ctx, d->gidx);
  d->d_own_src.upload(ctx, d->own_src);
  d->d_orig_src.upload(ctx, d->orig_src);
  d->d_orig_dst.upload(ctx, d->orig_dst);
  d->d_level_fronts.upload(ctx, lf);
  d->d_flf.upload(ctx, d->flf);
  d->w_total = wrows;
  d->d_imap.upload(ctx, imap);
  phase("  front descriptors, uploads");
  {  // solve worklists: forward row tiles of 64, backward column tiles of 32 (vector-unit
     // sweeps) and the wider tiles of the matrix-core sweeps.  Workgroups are dealt to the 8
     // XCDs round-robin by launch index, each XCD with its own L2.  All tiles of a front go to
     // one XCD, so the front's right-hand rows, which every tile reads, are fetched into one
     // L2 only.  Fronts are spread over the XCDs largest first onto the least-loaded one
     // (load = the tiles' factor entries), and the XCDs' lists are interleaved at stride 8
     // with (-1, 0) padding entries that exit at once.
    auto build = [&](int rows, int cols, std::vector<int64_t>& foff, std::vector<int64_t>& boff,
                     DevArray<int32_t>& dfw, DevArray<int32_t>& dbw) {
      constexpr int kXcd = 8;
      std::vector<int32_t> fw, bw;
      using Item = std::pair<int32_t, int32_t>;
      auto deal = [&](const std::vector<std::pair<double, std::vector<Item>>>& per_front, std::vector<int32_t>& out) {
        std::vector<std::vector<Item>> bins(kXcd);
        std::vector<double> load(kXcd, 0.0);
        std::vector<size_t> order(per_front.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t a, size_t b) { return per_front[a].first > per_front[b].first; });
        for (size_t k : order) {
          const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
          load[x] += per_front[k].first;
          bins[x].insert(bins[x].end(), per_front[k].second.begin(), per_front[k].second.end());
        }
        size_t mx = 0;
        for (auto& b : bins) mx = std::max(mx, b.size());
        for (size_t k = 0; k < mx; ++k)
          for (int x = 0; x < kXcd; ++x) {
            const Item it = k < bins[x].size() ? bins[x][k] : Item(-1, 0);
            out.push_back(it.first);
            out.push_back(it.second);
          }
      };
      for (const Level& L : d->levels) {
        foff.push_back((int64_t)fw.size() / 2);
        boff.push_back((int64_t)bw.size() / 2);
        std::vector<std::pair<double, std::vector<Item>>> pf, pb;
        for (int32_t fi : L.fronts) {
          const Front& F = d->fronts[fi];
          std::pair<double, std::vector<Item>> a, b;
          for (int64_t i0 = 0; i0 < F.f(); i0 += rows) {  // a row tile reads columns [0, min(p, i0 + rows))
            a.second.emplace_back(fi, (int32_t)i0);
            a.first += (double)std::min<int64_t>(rows, F.f() - i0) * (double)(i0 < F.p ? std::min<int64_t>(F.p, i0 + rows) : F.p);
          }
          for (int64_t j0 = 0; j0 < F.p; j0 += cols) {  // a column tile reads rows [j0, f)
            b.second.emplace_back(fi, (int32_t)j0);
            b.first += (double)std::min<int64_t>(cols, F.p - j0) * (double)(F.f() - j0);
          }
          pf.push_back(std::move(a));
          pb.push_back(std::move(b));
        }
        deal(pf, fw);
        deal(pb, bw);
      }
      foff.push_back((int64_t)fw.size() / 2);
      boff.push_back((int64_t)bw.size() / 2);
      dfw.upload(ctx, fw);
      dbw.upload(ctx, bw);
    };
    build(64, 32, d->fwd_off, d->bwd_off, d->d_fwd_work, d->d_bwd_work);
    for (int t = 0; t < 2; ++t)  // the matrix-core sweeps' tiles (both precisions)
      build(kFwdRowsMfma[t], kBwdColsMfma[t], d->fwdm_off[t], d->bwdm_off[t], d->d_fwdm_work[t], d->d_bwdm_work[t]);
  }
  {
    phase("  solve worklists");
    // concatenated local CSR patterns, Dirichlet flags, and what the device fill of the local
    // values reads: each subdomain's row incidences, tets, Robin masks and local-to-global map
    // (one subdomain per task)
    std::vector<int64_t> ioff(n_sub + 1, 0), toff(n_sub + 1, 0);
    for (int32_t i = 0; i < n_sub; ++i) {
      ioff[i + 1] = ioff[i] + (int64_t)d->subs[i].inc.idx.size();
      toff[i + 1] = toff[i] + (int64_t)d->subs[i].tsel.size();
    }
    std::vector<int64_t> rp(rows), ip(rows);
    std::vector<int32_t> cl(csr), ix(ioff[n_sub]), ts(toff[n_sub]), gd(vec);
    std::vector<uint8_t> dr(vec), rb(toff[n_sub]);
    each_sub([&](int32_t i) {
      const Subdomain& S = d->subs[i];
      std::copy(S.rowptr.begin(), S.rowptr.begin() + S.n + 1, rp.begin() + S.row_off);
      std::copy(S.inc.ptr.begin(), S.inc.ptr.begin() + S.n + 1, ip.begin() + S.row_off);
      std::copy(S.col.begin(), S.col.end(), cl.begin() + S.csr_off);
      std::copy(S.inc.idx.begin(), S.inc.idx.end(), ix.begin() + ioff[i]);
      std::copy(S.tsel.begin(), S.tsel.end(), ts.begin() + toff[i]);
      std::copy(S.robin.begin(), S.robin.end(), rb.begin() + toff[i]);
      std::copy(S.gdofs.begin(), S.gdofs.end(), gd.begin() + S.vec_off);
      std::copy(S.dir.begin(), S.dir.end(), dr.begin() + S.vec_off);
    });
    d->d_lrowptr.upload(ctx, rp);
    d->d_lcol.upload(ctx, cl);
    d->d_ldir.upload(ctx, dr);
    d->d_lval.alloc(ctx, csr);
    DevArray<int64_t> d_ip;
    DevArray<int32_t> d_ix, d_ts, d_gd;
    DevArray<uint8_t> d_rb;
    d_ip.upload(ctx, ip);
    d_ix.upload(ctx, ix);
    d_ts.upload(ctx, ts);
    d_rb.upload(ctx, rb);
    d_gd.upload(ctx, gd);
    phase("  local patterns, uploads");
    // element matrices of the operator (released after hz_assemble; the same kernel on the same
    // coefficients gives the same bits), kept only while the local operators are filled
    DevArray<double> dv, dq;
    dv.upload(ctx, op->velocity);
    if (op->has_q) dq.upload(ctx, op->Q);
    op->d_elem.alloc(ctx, m.T * kElemStride);
    launch_element_matrices(ctx, m, *op, dv.ptr(), op->has_q ? dq.ptr() : nullptr);
    // one launch per subdomain (row pointers are subdomain-relative)
    for (int32_t i = 0; i < n_sub; ++i) {
      const Subdomain& S = d->subs[i];
      launch_incidence_fill(ctx->stream, S.n, d->d_lrowptr.ptr() + S.row_off, d->d_lcol.ptr() + S.csr_off,
                            d_gd.ptr() + S.vec_off, d_ip.ptr() + S.row_off, d_ix.ptr() + ioff[i],
                            d_ts.ptr() + toff[i], d_rb.ptr() + toff[i], m.d_tet_dofs.ptr(), op->d_elem.ptr(),
                            d->d_ldir.ptr() + S.vec_off, d->d_lval.ptr() + S.csr_off, nullptr);
    }
    // the local values are assembled: what only their fill needed goes (host and device)
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
  }
  for (auto& S : d->subs) {
    S.inc = RowIncidence();
    S.tsel = std::vector<int32_t>();
    S.robin = std::vector<uint8_t>();
  }
  op->d_elem = DevArray<c128>();
  phase("device maps, local operators");
  // --- numeric factorisation; its algorithmic work per front (p pivots, f rows, panels of 32):
  // LDL^T of the p x p block (p^3 / 6), panel solves below it (sum over panels of
  // (f - k0 - nb) nb^2 / 2), trailing updates of the lower triangle (sum over panels of
  // (f - k0 - nb)^2 nb / 2), and the partitioned inverse (p^2 (f - p) / 2 + p^3 / 6): complex
  // multiply-adds, 8 real flops each
  {
    double cm = 0;
    for (const Front& F : d->fronts) {
      const double p = (double)F.p, f = (double)F.f();
      cm += p * p * p / 6.0 + p * p * (f - p) / 2.0 + p * p * p / 6.0;
      for (int64_t k0 = 0; k0 < F.p; k0 += 32) {
        const double nb = (double)std::min<int64_t>(32, F.p - k0), rem = f - (double)k0 - nb;
        cm += rem * nb * nb / 2.0 + rem * rem * nb / 2.0;
      }
    }
    d->factor_flops = 8.0 * cm;
  }
  if (local_solver != HZ_LOCAL_EXACT) {
    // the incomplete factors replace the exact ones (whose symbolic size stays reported)
    icc_setup(ctx, *d);
    phase("incomplete factorisation");
  } else {
    const double tf0 = wall_time();
    factor_all(ctx, *d);
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    d->factor_seconds = wall_time() - tf0;
    phase("numeric factorisation");
  }
  // set-up-only data: the scatter lists, and the local operator values unless small enough to
  // keep for introspection (hz_get_subdomain)
  d->d_orig_src = DevArray<int64_t>();
  d->d_orig_dst = DevArray<int64_t>();
  std::vector<int64_t>().swap(d->orig_src);
  std::vector<int64_t>().swap(d->orig_dst);
  if (d->d_lval.bytes() > (size_t(2) << 30)) d->d_lval = DevArray<c128>();
  // --- coarse space
  if (coarse) {
    d->coarse = std::make_unique<CoarseSpace>();
    build_coarse_host(m, coarse, *d->coarse);
    phase("coarse space (host)");
    coarse_setup(ctx, *d);
  }
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  phase("coarse space (device)");
  d->setup_seconds = wall_time() - t0;
  return d;
}

}  // namespace hz
