// Mesh ingest: P3 dof numbering, face neighbours, boundary tags, Dirichlet dofs, CSR
// pattern and the deterministic gather map used by the assembly kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <functional>
#include <thread>

#include "hz_internal.h"

namespace hz {

double wall_time() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body) {
  int nt = (int)std::min<int64_t>(std::max(1u, std::thread::hardware_concurrency()), 16);
  if (n < 4096 || nt == 1) {
    body(0, n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([&, a, b] { body(a, b); });
  }
  for (auto& x : th) x.join();
}

namespace {

const int kEdges[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

struct Key {
  uint64_t hi, lo;
  uint32_t idx;
};
inline bool key_less(const Key& a, const Key& b) { return a.hi != b.hi ? a.hi < b.hi : a.lo < b.lo; }

// barycentric weights of the 20 local nodes
void node_weights(double w[20][4]) {
  for (int i = 0; i < 20; ++i)
    for (int v = 0; v < 4; ++v) w[i][v] = 0;
  for (int v = 0; v < 4; ++v) w[v][v] = 1;
  for (int e = 0; e < 6; ++e) {
    int a = kEdges[e][0], b = kEdges[e][1];
    w[4 + 2 * e][a] = 2.0 / 3.0;
    w[4 + 2 * e][b] = 1.0 / 3.0;
    w[5 + 2 * e][a] = 1.0 / 3.0;
    w[5 + 2 * e][b] = 2.0 / 3.0;
  }
  for (int f = 0; f < 4; ++f)
    for (int v = 0; v < 4; ++v)
      if (v != f) w[16 + f][v] = 1.0 / 3.0;
}

}  // namespace

std::shared_ptr<Mesh> build_mesh(Ctx* ctx, int64_t T, const int32_t* tets, int64_t V, const double* coords,
                                 const int8_t* face_bc) {
  HZ_REQUIRE(T > 0 && V >= 4 && tets && coords, HZ_ERR_ARG, "hz_mesh: empty mesh or null pointer");
  HZ_REQUIRE(T * 20 < (int64_t)UINT32_MAX, HZ_ERR_ARG, "hz_mesh: too many tets");
  auto m = std::make_shared<Mesh>();
  m->T = T;
  m->V = V;
  m->tets.assign(tets, tets + 4 * T);
  m->coords.assign(coords, coords + 3 * V);
  for (int64_t i = 0; i < 4 * T; ++i)
    HZ_REQUIRE(m->tets[i] >= 0 && m->tets[i] < V, HZ_ERR_ARG, "hz_mesh: vertex id out of range");
  for (int64_t i = 0; i < 3 * V; ++i) HZ_REQUIRE(std::isfinite(m->coords[i]), HZ_ERR_ARG, "hz_mesh: non-finite coordinate");
  for (int64_t t = 0; t < T; ++t) {
    const int32_t* tv = &m->tets[4 * t];
    HZ_REQUIRE(tv[0] != tv[1] && tv[0] != tv[2] && tv[0] != tv[3] && tv[1] != tv[2] && tv[1] != tv[3] && tv[2] != tv[3],
               HZ_ERR_ARG, "hz_mesh: repeated vertex in a tet");
  }

  // --- dof keys and ranks
  std::vector<Key> keys(T * 20);
  parallel_for(T, [&](int64_t a, int64_t b) {
    for (int64_t t = a; t < b; ++t) {
      const int32_t* tv = &m->tets[4 * t];
      auto put = [&](int l, int64_t v0, int64_t v1, int64_t v2, int sub) {
        Key& k = keys[t * 20 + l];
        k.hi = ((uint64_t)v0 << 32) | (uint64_t)(uint32_t)(v1 + 1);
        k.lo = ((uint64_t)(uint32_t)(v2 + 1) << 1) | (uint64_t)sub;
        k.idx = (uint32_t)(t * 20 + l);
      };
      for (int v = 0; v < 4; ++v) put(v, tv[v], -1, -1, 0);
      for (int e = 0; e < 6; ++e) {
        int64_t ga = tv[kEdges[e][0]], gb = tv[kEdges[e][1]];
        int64_t lo = std::min(ga, gb), hi = std::max(ga, gb);
        bool a_lo = ga < gb;
        put(4 + 2 * e, lo, hi, -1, a_lo ? 0 : 1);  // node nearer a
        put(5 + 2 * e, lo, hi, -1, a_lo ? 1 : 0);  // node nearer b
      }
      for (int f = 0; f < 4; ++f) {
        int64_t s[3];
        int c = 0;
        for (int v = 0; v < 4; ++v)
          if (v != f) s[c++] = tv[v];
        std::sort(s, s + 3);
        put(16 + f, s[0], s[1], s[2], 0);
      }
    }
  });
  std::sort(keys.begin(), keys.end(), key_less);
  m->tet_dofs.assign(T * 20, 0);
  int64_t n = 0;
  for (size_t i = 0; i < keys.size(); ++i) {
    if (i > 0 && (keys[i].hi != keys[i - 1].hi || keys[i].lo != keys[i - 1].lo)) ++n;
    m->tet_dofs[keys[i].idx] = (int32_t)n;
  }
  m->n = n + 1;
  HZ_REQUIRE(m->n < INT32_MAX, HZ_ERR_ARG, "hz_mesh: too many dofs");
  keys.clear();
  keys.shrink_to_fit();

  // --- face neighbours
  std::vector<Key> fk(T * 4);
  parallel_for(T, [&](int64_t a, int64_t b) {
    for (int64_t t = a; t < b; ++t) {
      const int32_t* tv = &m->tets[4 * t];
      for (int f = 0; f < 4; ++f) {
        int64_t s[3];
        int c = 0;
        for (int v = 0; v < 4; ++v)
          if (v != f) s[c++] = tv[v];
        std::sort(s, s + 3);
        Key& k = fk[t * 4 + f];
        k.hi = ((uint64_t)s[0] << 32) | (uint64_t)s[1];
        k.lo = (uint64_t)s[2];
        k.idx = (uint32_t)(t * 4 + f);
      }
    }
  });
  std::sort(fk.begin(), fk.end(), key_less);
  m->nbr.assign(T * 4, -1);
  for (size_t i = 0; i + 1 < fk.size(); ++i) {
    if (fk[i].hi == fk[i + 1].hi && fk[i].lo == fk[i + 1].lo) {
      HZ_REQUIRE(i + 2 >= fk.size() || fk[i + 2].hi != fk[i].hi || fk[i + 2].lo != fk[i].lo, HZ_ERR_ARG,
                 "hz_mesh: a face is shared by more than two tets");
      m->nbr[fk[i].idx] = fk[i + 1].idx / 4;
      m->nbr[fk[i + 1].idx] = fk[i].idx / 4;
      ++i;
    }
  }
  fk.clear();
  fk.shrink_to_fit();

  // --- boundary tags and Dirichlet dofs
  const P3Tables& tab = p3_tables();
  m->tag.assign(T * 4, HZ_BC_NONE);
  m->dirichlet.assign(m->n, 0);
  for (int64_t t = 0; t < T; ++t)
    for (int f = 0; f < 4; ++f) {
      if (m->nbr[t * 4 + f] >= 0) continue;
      int8_t tg = face_bc ? face_bc[t * 4 + f] : (int8_t)HZ_BC_IMPEDANCE;
      HZ_REQUIRE(tg == HZ_BC_IMPEDANCE || tg == HZ_BC_DIRICHLET, HZ_ERR_ARG, "hz_mesh: invalid boundary tag");
      m->tag[t * 4 + f] = tg;
      if (tg == HZ_BC_DIRICHLET)
        for (int a = 0; a < 10; ++a) m->dirichlet[m->tet_dofs[t * 20 + tab.face_nodes[f][a]]] = 1;
    }

  // --- dof coordinates and element sanity
  double w[20][4];
  node_weights(w);
  m->dof_xyz.assign(3 * m->n, 0.0);
  for (int64_t t = 0; t < T; ++t) {
    const int32_t* tv = &m->tets[4 * t];
    const double* p0 = &m->coords[3 * tv[0]];
    double J[3][3];
    for (int c = 0; c < 3; ++c)
      for (int d = 0; d < 3; ++d) J[d][c] = m->coords[3 * tv[c + 1] + d] - p0[d];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    HZ_REQUIRE(det != 0.0 && std::isfinite(det), HZ_ERR_ARG, "hz_mesh: degenerate tet");
    for (int l = 0; l < 20; ++l) {
      int32_t g = m->tet_dofs[t * 20 + l];
      for (int d = 0; d < 3; ++d) {
        double x = 0;
        for (int v = 0; v < 4; ++v) x += w[l][v] * m->coords[3 * tv[v] + d];
        m->dof_xyz[3 * g + d] = x;
      }
    }
  }

  // --- device copies
  m->d_tets.upload(ctx, m->tets);
  m->d_coords.upload(ctx, m->coords);
  m->d_tet_dofs.upload(ctx, m->tet_dofs);
  m->d_dirichlet.upload(ctx, m->dirichlet);
  return m;
}

void build_pattern_and_incidence(const Mesh& m, const std::vector<int64_t>& tets_sel, const std::vector<int32_t>& loc,
                                 int64_t n_local, std::vector<int64_t>& rowptr, std::vector<int32_t>& col,
                                 RowIncidence& inc) {
  const int64_t Ts = (int64_t)tets_sel.size();
  HZ_REQUIRE(Ts * 20 < (int64_t)INT32_MAX, HZ_ERR_ARG, "assembly: too many tets in one operator");
  // local dof -> (selected tet position, node) in ascending tet order
  inc.ptr.assign(n_local + 1, 0);
  for (int64_t q = 0; q < Ts; ++q)
    for (int l = 0; l < 20; ++l) {
      int32_t r = loc[m.tet_dofs[tets_sel[q] * 20 + l]];
      HZ_REQUIRE(r >= 0 && r < n_local, HZ_ERR_STATE, "pattern: dof outside local numbering");
      inc.ptr[r + 1]++;
    }
  for (int64_t r = 0; r < n_local; ++r) inc.ptr[r + 1] += inc.ptr[r];
  inc.idx.resize(inc.ptr[n_local]);
  {
    std::vector<int64_t> fill(inc.ptr.begin(), inc.ptr.end() - 1);
    for (int64_t q = 0; q < Ts; ++q)
      for (int l = 0; l < 20; ++l) {
        int32_t r = loc[m.tet_dofs[tets_sel[q] * 20 + l]];
        inc.idx[fill[r]++] = (int32_t)(q * 20 + l);
      }
  }
  // pattern
  rowptr.assign(n_local + 1, 0);
  std::vector<std::vector<int32_t>> rows(n_local);
  parallel_for(n_local, [&](int64_t a, int64_t b) {
    std::vector<int32_t> buf;
    for (int64_t r = a; r < b; ++r) {
      buf.clear();
      for (int64_t k = inc.ptr[r]; k < inc.ptr[r + 1]; ++k) {
        int64_t q = inc.idx[k] / 20;
        for (int j = 0; j < 20; ++j) buf.push_back(loc[m.tet_dofs[tets_sel[q] * 20 + j]]);
      }
      std::sort(buf.begin(), buf.end());
      buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
      rows[r] = buf;
    }
  });
  for (int64_t r = 0; r < n_local; ++r) rowptr[r + 1] = rowptr[r] + (int64_t)rows[r].size();
  col.resize(rowptr[n_local]);
  parallel_for(n_local, [&](int64_t a, int64_t b) {
    for (int64_t r = a; r < b; ++r) std::copy(rows[r].begin(), rows[r].end(), col.begin() + rowptr[r]);
  });
}

}  // namespace hz
