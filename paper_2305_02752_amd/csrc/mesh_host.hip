// Mesh validation and rest-state construction on the host.
#include <algorithm>
#include <cmath>
#include <map>

#include "host.h"

namespace hc {

std::string build_mesh(const hc_mesh_desc* d, HostMesh& m) {
  if (!d || !d->tri || !d->rest_pos) return "mesh: null pointer";
  const int nv = d->n_vert, nt = d->n_tri;
  if (nv < 2 * kNPole || nt < 4) return "mesh: need >= 64 vertices and >= 4 triangles";
  m.nv = nv;
  m.nt = nt;
  m.tri.assign(d->tri, d->tri + 3 * nt);
  std::vector<double> X(d->rest_pos, d->rest_pos + 3 * nv);
  auto P = [&](int i, int k) { return X[3 * i + k]; };
  // directed edge -> (triangle, wing vertex)
  std::map<std::pair<int, int>, std::pair<int, int>> dir;
  for (int t = 0; t < nt; ++t) {
    for (int r = 0; r < 3; ++r) {
      const int a = m.tri[3 * t + r], b = m.tri[3 * t + (r + 1) % 3], w = m.tri[3 * t + (r + 2) % 3];
      if (a < 0 || a >= nv || b < 0 || b >= nv || w < 0 || w >= nv) return "mesh: index out of range";
      if (!dir.emplace(std::make_pair(a, b), std::make_pair(t, w)).second)
        return "mesh: repeated directed edge (inconsistent orientation)";
    }
  }
  std::vector<int> degree(nv, 0);
  for (auto& kv : dir) {
    const int p = kv.first.first, q = kv.first.second;
    auto rev = dir.find(std::make_pair(q, p));
    if (rev == dir.end()) return "mesh: open edge (surface not closed)";
    ++degree[p];
    if (p < q) {
      const int k = kv.second.second, l = rev->second.second;
      double s = 0;
      for (int a = 0; a < 3; ++a) s += (P(q, a) - P(p, a)) * (P(q, a) - P(p, a));
      m.edge.insert(m.edge.end(), {p, q});
      m.L0.push_back((float)std::sqrt(s));
      m.hinge_v.insert(m.hinge_v.end(), {p, q, k, l});
      // rest dihedral angle, float64
      double e[3], u1[3], v1[3], u2[3], v2[3], n1[3], n2[3];
      for (int a = 0; a < 3; ++a) {
        e[a] = P(q, a) - P(p, a);
        u1[a] = e[a];
        v1[a] = P(k, a) - P(p, a);
        u2[a] = P(p, a) - P(q, a);
        v2[a] = P(l, a) - P(q, a);
      }
      auto cr = [](const double* a, const double* b, double* o) {
        o[0] = a[1] * b[2] - a[2] * b[1];
        o[1] = a[2] * b[0] - a[0] * b[2];
        o[2] = a[0] * b[1] - a[1] * b[0];
      };
      cr(u1, v1, n1);
      cr(u2, v2, n2);
      auto nrm = [](double* a) {
        const double s = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        a[0] /= s; a[1] /= s; a[2] /= s;
      };
      nrm(n1);
      nrm(n2);
      nrm(e);
      double x[3];
      cr(n1, n2, x);
      const double sn = x[0] * e[0] + x[1] * e[1] + x[2] * e[2];
      const double cs = n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2];
      m.theta0.push_back((float)std::atan2(sn, cs));
    }
  }
  for (int v = 0; v < nv; ++v)
    if (degree[v] == 0) return "mesh: isolated vertex";
  m.ne = (int)m.L0.size();
  m.nh = m.ne;
  // each triangle is evaluated with one hinge of its first stored edge (a, b):
  // bit 0 when it is that hinge's (i, j, k) (a < b), bit 1 its (j, i, l)
  {
    std::map<std::pair<int, int>, int> hidx;
    for (int h = 0; h < m.nh; ++h) hidx[std::make_pair(m.hinge_v[4 * h], m.hinge_v[4 * h + 1])] = h;
    m.hinge_own.assign(m.nh, 0);
    for (int t = 0; t < nt; ++t) {
      const int a = m.tri[3 * t], b = m.tri[3 * t + 1];
      const int h = hidx.at(std::make_pair(std::min(a, b), std::max(a, b)));
      m.hinge_own[h] |= a < b ? 1 : 2;
    }
  }
  // rest area and volume (float64, divergence theorem)
  double A = 0, V = 0;
  for (int t = 0; t < nt; ++t) {
    const int a = m.tri[3 * t], b = m.tri[3 * t + 1], c = m.tri[3 * t + 2];
    double u[3], w[3], n[3];
    for (int k = 0; k < 3; ++k) {
      u[k] = P(b, k) - P(a, k);
      w[k] = P(c, k) - P(a, k);
    }
    n[0] = u[1] * w[2] - u[2] * w[1];
    n[1] = u[2] * w[0] - u[0] * w[2];
    n[2] = u[0] * w[1] - u[1] * w[0];
    A += 0.5 * std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    V += (P(a, 0) * (P(b, 1) * P(c, 2) - P(b, 2) * P(c, 1)) +
          P(a, 1) * (P(b, 2) * P(c, 0) - P(b, 0) * P(c, 2)) +
          P(a, 2) * (P(b, 0) * P(c, 1) - P(b, 1) * P(c, 0))) / 6.0;
  }
  if (!(V > 0)) return "mesh: non-positive volume (triangles must be counter-clockwise from outside)";
  m.A0 = A;
  m.V0 = V;
  // traction poles: 32 largest / smallest rest x, ties to the lower index
  std::vector<int> idx(nv);
  for (int i = 0; i < nv; ++i) idx[i] = i;
  m.pole.assign(nv, 0.f);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return P(a, 0) > P(b, 0); });
  for (int i = 0; i < kNPole; ++i) m.pole[idx[i]] = 1.f;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return P(a, 0) < P(b, 0); });
  for (int i = 0; i < kNPole; ++i) {
    if (m.pole[idx[i]] != 0.f) return "mesh: pole sets overlap";
    m.pole[idx[i]] = -1.f;
  }
  return "";
}

}  // namespace hc
