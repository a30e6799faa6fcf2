// TEST INFRASTRUCTURE -- CPU oracle for the volumetric restricted power diagram (RPD) with fractional Euler
// characteristics and connected components. Only the test-suite, the smoke entry point and the benchmark's
// CPU-baseline leg may load this library; the product path never does. It shares no code with the GPU path.
//
// What it computes (paper: Sec. 3.2 power cell / RPD definitions, Sec. 3.3 nerve and contractibility,
// Sec. 4.1.1 connected components, Sec. 4.1.2 fractional Euler characteristic, Sec. 5.2 Tet-Cell clipping):
//
//   * power distance d_i(x) = |x - c_i|^2 - r_i^2; closed power cell Omega_i = {x : d_i(x) <= d_j(x) for all j};
//     restricted cell RPC_i = Omega_i intersected with the tet mesh S; RPF_ij = RPC_i & RPC_j; RPE_ijk; RPV_ijkl.
//   * For every tet t and EVERY site i (brute force, all sites), the piece P_{t,i} = t & Omega_i is obtained by
//     clipping t successively by the half-spaces H_ij = {d_i <= d_j} of ALL other sites j (any order; nearest first
//     here so that empty pieces stop early). Every sign is decided exactly with integer arithmetic.
//   * Fractional Euler characteristic (Sec. 4.1.2): each mesh simplex sigma carries weight 1/k(sigma), k(sigma)
//     = number of tets containing it; an element of a piece inherits the weight of its carrier (the mesh simplex
//     whose relative interior contains it); elements interior to a tet weigh 1. Stored as integers over
//     L = lcm of all k(sigma).  chi(RPC) = V - E + F - C, chi(RPF) = V - E + F, chi(RPE) = V - E (signs by the
//     element's own dimension, following the paper's worked example).
//   * Explicit assembly: the same chi counted as an integer V - E + F - C over globally merged keys (carrier,
//     site set); the oracle checks that both agree.
//   * beta0: union-find over pieces glued through 2D contact on a shared mesh face (cells), 1D contact on a
//     shared mesh face (faces) and a point on a shared mesh face (edges); checked against 1-skeleton
//     connectivity of the assembled complex.
//   * volume and centroid of every RPC (Lebesgue measure / first moment over S), FP64.
//
//   * Ownership weights (meshes whose lcm of multiplicities reaches 2^31, or on request): each mesh simplex sigma
//     weighs 1 in its owner tet, the lowest-numbered tet containing it, and 0 in the others, with L = 1. Summed over
//     the tets around sigma this is the same total weight 1 as k(sigma) times 1/k(sigma), so every element's chi is
//     unchanged; only its split over the pieces differs.
//
//   * Exact ties (a vertex exactly on a clipping plane: a bisector through a mesh vertex, five co-spherical sites,
//     equal spheres) are broken by symbolic perturbation of the weights (simulation of simplicity): site s's squared
//     radius becomes W_s + eps_s with eps_0 >> eps_1 >> ... > 0, so a lower site id wins a tie.
//
// Readings of the paper (where it is silent): weights w(sigma)=1/k(sigma) generalise the 2D example; ties as
// above (the paper assumes a clean cut); empty cells report chi=0,
// beta0=0, volume 0 and a NaN centroid.
//
// Inputs are float32 values on the 2^-20 grid; they are converted exactly to integers in units of 2^-20.

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

typedef int64_t i64;
typedef __int128 i128;
typedef unsigned __int128 u128;

namespace {

// ---------------------------------------------------------------------------------------------------------------
// 256-bit two's complement integers (4 x 64-bit limbs), enough for every determinant below.
// ---------------------------------------------------------------------------------------------------------------
struct I256 {
  uint64_t w[4];
};

I256 from128(i128 v) {
  I256 r;
  r.w[0] = (uint64_t)v;
  r.w[1] = (uint64_t)((u128)v >> 64);
  uint64_t s = v < 0 ? ~0ull : 0ull;
  r.w[2] = s;
  r.w[3] = s;
  return r;
}

I256 add(const I256& a, const I256& b) {
  I256 r;
  u128 c = 0;
  for (int k = 0; k < 4; ++k) {
    c += (u128)a.w[k] + b.w[k];
    r.w[k] = (uint64_t)c;
    c >>= 64;
  }
  return r;
}

I256 neg(const I256& a) {
  I256 r;
  u128 c = 1;
  for (int k = 0; k < 4; ++k) {
    c += (u128)(~a.w[k]);
    r.w[k] = (uint64_t)c;
    c >>= 64;
  }
  return r;
}

I256 sub(const I256& a, const I256& b) { return add(a, neg(b)); }

bool isneg(const I256& a) { return (a.w[3] >> 63) != 0; }

I256 mul(I256 a, I256 b) {
  bool na = isneg(a), nb = isneg(b);
  if (na) a = neg(a);
  if (nb) b = neg(b);
  I256 r = {{0, 0, 0, 0}};
  for (int i = 0; i < 4; ++i) {
    u128 carry = 0;
    for (int j = 0; i + j < 4; ++j) {
      u128 t = (u128)a.w[i] * b.w[j] + r.w[i + j] + carry;
      r.w[i + j] = (uint64_t)t;
      carry = t >> 64;
    }
  }
  return na != nb ? neg(r) : r;
}

int sgn(const I256& a) {
  if (isneg(a)) return -1;
  return (a.w[0] | a.w[1] | a.w[2] | a.w[3]) ? 1 : 0;
}

long double to_ld(const I256& a0) {
  bool n = isneg(a0);
  I256 a = n ? neg(a0) : a0;
  long double r = 0;
  for (int k = 3; k >= 0; --k) r = r * 18446744073709551616.0L + (long double)a.w[k];
  return n ? -r : r;
}

// ---------------------------------------------------------------------------------------------------------------
// Planes in integer tet-local coordinates Y = X - O (X in units of 2^-20, O = the tet's first vertex):
// plane(Y) = n . Y + d, the kept side is plane(Y) >= 0.
// ---------------------------------------------------------------------------------------------------------------
struct Plane {
  i128 n[3];
  i128 d;
  int kind;  // 0 = tet face (id = local face index f, the face opposite local vertex f), 1 = bisector (id = site)
  int id;
};

// det3 of three normals as a 256-bit integer: a . (b x c)
I256 det3(const i128* a, const i128* b, const i128* c) {
  i128 x = b[1] * c[2] - b[2] * c[1];
  i128 y = b[2] * c[0] - b[0] * c[2];
  i128 z = b[0] * c[1] - b[1] * c[0];
  I256 r = mul(from128(a[0]), from128(x));
  r = add(r, mul(from128(a[1]), from128(y)));
  r = add(r, mul(from128(a[2]), from128(z)));
  return r;
}

// Sign of plane q at the point where planes a, b, c meet.  With M = det[[n_a d_a];[n_b d_b];[n_c d_c];[n_q d_q]]
// and Delta = det[n_a; n_b; n_c], the value of plane q at that point equals M / Delta (Cramer's rule on the
// homogeneous system), so its sign is sign(M) * sign(Delta).
I256 side_value(const Plane& a, const Plane& b, const Plane& c, const Plane& q, int* sd_out) {
  I256 m_a = det3(b.n, c.n, q.n);
  I256 m_b = det3(a.n, c.n, q.n);
  I256 m_c = det3(a.n, b.n, q.n);
  I256 m_q = det3(a.n, b.n, c.n);
  // cofactor expansion of M along the d column: -d_a m_a + d_b m_b - d_c m_c + d_q m_q
  I256 M = mul(from128(q.d), m_q);
  M = sub(M, mul(from128(a.d), m_a));
  M = add(M, mul(from128(b.d), m_b));
  M = sub(M, mul(from128(c.d), m_c));
  *sd_out = sgn(m_q);
  return M;
}

int side_exact(const Plane& a, const Plane& b, const Plane& c, const Plane& q, int* delta_zero) {
  int sd = 0;
  I256 M = side_value(a, b, c, q, &sd);
  if (delta_zero) *delta_zero = (sd == 0);
  return sgn(M) * sd;
}

// The same sign with exact zeros broken by symbolic perturbation of the weights: site s's squared radius becomes
// W_s + eps_s, eps_0 >> eps_1 >> ... > 0 infinitesimal, so a bisector of the cell's site si against site j gains
// eps_si - eps_j in its offset (power distance of the origin to j minus that to si) and face planes do not move.
// The value M is linear in the four offsets, so the coefficient of eps_s is the change of M when s's weight
// grows by one unit; the sign is that of the first nonzero coefficient in increasing site order.
int side_sos(const Plane& a, const Plane& b, const Plane& c, const Plane& q, int si, int* delta_zero) {
  int sd = 0;
  I256 M = side_value(a, b, c, q, &sd);
  *delta_zero = (sd == 0);
  if (sd == 0 || sgn(M) != 0) return sgn(M) * sd;
  const Plane* pl[4] = {&a, &b, &c, &q};
  std::vector<int> sites = {si};
  for (const Plane* p : pl)
    if (p->kind == 1) sites.push_back(p->id);
  std::sort(sites.begin(), sites.end());
  sites.erase(std::unique(sites.begin(), sites.end()), sites.end());
  for (int s : sites) {
    Plane moved[4] = {a, b, c, q};
    for (Plane& p : moved)
      if (p.kind == 1) p.d += (s == si ? 1 : 0) - (s == p.id ? 1 : 0);
    int sd2 = 0;
    I256 coef = sub(side_value(moved[0], moved[1], moved[2], moved[3], &sd2), M);
    if (sgn(coef) != 0) return sgn(coef) * sd;
  }
  return 0;
}

// Exact point of three planes (as long double coordinates, tet-local, units 2^-20):
// Y = -(d_a (n_b x n_c) + d_b (n_c x n_a) + d_c (n_a x n_b)) / Delta
void point3(const Plane& a, const Plane& b, const Plane& c, long double out[3]) {
  auto cross = [](const i128* u, const i128* v, i128* r) {
    r[0] = u[1] * v[2] - u[2] * v[1];
    r[1] = u[2] * v[0] - u[0] * v[2];
    r[2] = u[0] * v[1] - u[1] * v[0];
  };
  i128 bc[3], ca[3], ab[3];
  cross(b.n, c.n, bc);
  cross(c.n, a.n, ca);
  cross(a.n, b.n, ab);
  I256 delta = det3(a.n, b.n, c.n);
  long double dl = to_ld(delta);
  for (int k = 0; k < 3; ++k) {
    I256 num = mul(from128(a.d), from128(bc[k]));
    num = add(num, mul(from128(b.d), from128(ca[k])));
    num = add(num, mul(from128(c.d), from128(ab[k])));
    out[k] = -to_ld(num) / dl;
  }
}

// ---------------------------------------------------------------------------------------------------------------
// status codes (same meaning as the library's, defined independently)
// ---------------------------------------------------------------------------------------------------------------
enum { OK = 0, E_INVALID = -1, E_MESH = -2, E_DEGENERATE = -3, E_NOMEM = -4, E_INCONSISTENT = -10 };

struct Failure {
  int code;
  std::string msg;
};

// ---------------------------------------------------------------------------------------------------------------
// Mesh: integer vertices, tets, global simplex ids and k(sigma).
// ---------------------------------------------------------------------------------------------------------------
const int EDGE_V[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

int local_edge(int a, int b) {
  if (a > b) std::swap(a, b);
  for (int e = 0; e < 6; ++e)
    if (EDGE_V[e][0] == a && EDGE_V[e][1] == b) return e;
  return -1;
}

i64 gcd64(i64 a, i64 b) {
  while (b) {
    i64 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

struct Mesh {
  int nv = 0, nt = 0;
  std::vector<i64> X, Y, Z;              // grid integers
  std::vector<std::array<int, 4>> tv;    // tets
  std::vector<std::array<int, 6>> tedge; // global edge id of local edge e
  std::vector<std::array<int, 4>> tface; // global face id of local face f (opposite vertex f)
  std::vector<std::array<int, 4>> tnb;   // neighbour tet across local face f, -1 on the boundary
  std::vector<int> kv, ke, kf;           // k(sigma)
  std::vector<int> ov, oe, of;           // owner tet of each vertex, edge, face (ownership weights)
  bool own = false;                      // ownership weights instead of L / k(sigma)
  int n_edges = 0, n_faces = 0, n_used_verts = 0;
  i64 L = 1;
  int chi = 0;
  int components = 0;
};

bool grid_int(float x, i64* out) {
  if (!std::isfinite(x)) return false;
  double s = (double)x * 1048576.0;
  double r = std::nearbyint(s);
  if (r != s) return false;
  *out = (i64)r;
  return true;
}

int find_root(std::vector<int>& p, int x) {
  while (p[x] != x) {
    p[x] = p[p[x]];
    x = p[x];
  }
  return x;
}

void unite(std::vector<int>& p, int a, int b) {
  a = find_root(p, a);
  b = find_root(p, b);
  if (a == b) return;
  if (a < b) std::swap(a, b);
  p[a] = b;
}

// The input is a manifold tet mesh (Sec. 3.3, Assumption). Besides every face lying in one or two tets, the link of
// every edge must be a circle or an arc, and the link of every vertex a sphere or a disk:
//  - edge e: the tets containing e, joined through the faces that contain e and are shared by two tets, form one
//    connected chain;
//  - vertex v: the tets containing v, joined through the shared faces that contain v, are connected, and the link
//    surface (one triangle per tet, one edge per face and one vertex per edge containing v) has Euler characteristic
//    2 and no boundary (an interior vertex) or 1 and a boundary (a boundary vertex), i.e. it is a sphere or a disk.
void check_links(const Mesh& m) {
  std::vector<std::vector<int>> etets(m.n_edges), vtets(m.nv);
  for (int t = 0; t < m.nt; ++t) {
    for (int e = 0; e < 6; ++e) etets[m.tedge[t][e]].push_back(t);
    for (int k = 0; k < 4; ++k) vtets[m.tv[t][k]].push_back(t);
  }
  // connected components of a set of tets under the given face joins (faces identified by local index)
  auto one_piece = [&](const std::vector<int>& tets, auto face_joins) {
    std::map<int, int> idx;
    for (int t : tets) idx.emplace(t, (int)idx.size());
    std::vector<int> par(idx.size());
    std::iota(par.begin(), par.end(), 0);
    for (int t : tets)
      for (int f = 0; f < 4; ++f) {
        const int nb = m.tnb[t][f];
        if (nb >= 0 && face_joins(t, f)) unite(par, idx[t], idx.at(nb));
      }
    int roots = 0;
    for (size_t k = 0; k < par.size(); ++k)
      if (find_root(par, (int)k) == (int)k) ++roots;
    return roots == 1;
  };
  for (int t = 0; t < m.nt; ++t)
    for (int e = 0; e < 6; ++e) {
      const int id = m.tedge[t][e];
      if (etets[id].empty()) continue;  // checked once, from its first tet
      const int a = m.tv[t][EDGE_V[e][0]], b = m.tv[t][EDGE_V[e][1]];
      // a face of tet u contains {a, b} iff the vertex opposite it is neither a nor b
      bool ok = one_piece(etets[id], [&](int u, int f) { return m.tv[u][f] != a && m.tv[u][f] != b; });
      if (!ok) throw Failure{E_MESH, "non-manifold edge: the tets around an edge are not one chain"};
      etets[id].clear();
    }
  for (int v = 0; v < m.nv; ++v) {
    if (vtets[v].empty()) continue;
    if (!one_piece(vtets[v], [&](int u, int f) { return m.tv[u][f] != v; }))
      throw Failure{E_MESH, "non-manifold vertex: the tets around a vertex are not connected"};
    std::set<int> edges, faces;
    bool boundary = false;
    for (int u : vtets[v]) {
      for (int e = 0; e < 6; ++e)
        if (m.tv[u][EDGE_V[e][0]] == v || m.tv[u][EDGE_V[e][1]] == v) edges.insert(m.tedge[u][e]);
      for (int f = 0; f < 4; ++f)
        if (m.tv[u][f] != v) {
          faces.insert(m.tface[u][f]);
          if (m.tnb[u][f] < 0) boundary = true;
        }
    }
    const long chi = (long)edges.size() - (long)faces.size() + (long)vtets[v].size();
    if (!((chi == 2 && !boundary) || (chi == 1 && boundary)))
      throw Failure{E_MESH, "non-manifold vertex: its link is not a sphere or a disk"};
  }
}

Mesh build_mesh(int nv, const float* vx, const float* vy, const float* vz, int nt, const int32_t* tv,
                bool force_owner) {
  Mesh m;
  if (nv <= 0 || nt <= 0) throw Failure{E_INVALID, "empty mesh"};
  m.nv = nv;
  m.nt = nt;
  m.X.resize(nv);
  m.Y.resize(nv);
  m.Z.resize(nv);
  for (int v = 0; v < nv; ++v) {
    if (!grid_int(vx[v], &m.X[v]) || !grid_int(vy[v], &m.Y[v]) || !grid_int(vz[v], &m.Z[v]))
      throw Failure{E_INVALID, "vertex coordinate not on the 2^-20 grid or not finite"};
    if (std::llabs(m.X[v]) > (1 << 20) || std::llabs(m.Y[v]) > (1 << 20) || std::llabs(m.Z[v]) > (1 << 20))
      throw Failure{E_INVALID, "vertex coordinate outside [-1,1]"};
  }
  m.tv.resize(nt);
  for (int t = 0; t < nt; ++t) {
    for (int k = 0; k < 4; ++k) {
      int v = tv[4 * t + k];
      if (v < 0 || v >= nv) throw Failure{E_INVALID, "tet vertex index out of range"};
      m.tv[t][k] = v;
    }
    const auto& q = m.tv[t];
    i128 ax = m.X[q[1]] - m.X[q[0]], ay = m.Y[q[1]] - m.Y[q[0]], az = m.Z[q[1]] - m.Z[q[0]];
    i128 bx = m.X[q[2]] - m.X[q[0]], by = m.Y[q[2]] - m.Y[q[0]], bz = m.Z[q[2]] - m.Z[q[0]];
    i128 cx = m.X[q[3]] - m.X[q[0]], cy = m.Y[q[3]] - m.Y[q[0]], cz = m.Z[q[3]] - m.Z[q[0]];
    i128 det = ax * (by * cz - bz * cy) - ay * (bx * cz - bz * cx) + az * (bx * cy - by * cx);
    if (det <= 0) throw Failure{E_INVALID, "tet not positively oriented"};
  }
  // global edges and faces via sorted keys
  std::map<std::pair<int, int>, int> emap;
  std::map<std::array<int, 3>, int> fmap;
  m.tedge.resize(nt);
  m.tface.resize(nt);
  m.tnb.assign(nt, {-1, -1, -1, -1});
  m.kv.assign(nv, 0);
  std::vector<std::vector<std::pair<int, int>>> face_tets;
  for (int t = 0; t < nt; ++t) {
    const auto& q = m.tv[t];
    for (int k = 0; k < 4; ++k) m.kv[q[k]]++;
    for (int e = 0; e < 6; ++e) {
      int a = q[EDGE_V[e][0]], b = q[EDGE_V[e][1]];
      if (a == b) throw Failure{E_INVALID, "repeated vertex in tet"};
      auto key = std::make_pair(std::min(a, b), std::max(a, b));
      auto it = emap.find(key);
      int id;
      if (it == emap.end()) {
        id = (int)emap.size();
        emap[key] = id;
        m.ke.push_back(0);
      } else {
        id = it->second;
      }
      m.ke[id]++;
      m.tedge[t][e] = id;
    }
    for (int f = 0; f < 4; ++f) {
      std::array<int, 3> key;
      int c = 0;
      for (int k = 0; k < 4; ++k)
        if (k != f) key[c++] = q[k];
      std::sort(key.begin(), key.end());
      auto it = fmap.find(key);
      int id;
      if (it == fmap.end()) {
        id = (int)fmap.size();
        fmap[key] = id;
        m.kf.push_back(0);
        face_tets.emplace_back();
      } else {
        id = it->second;
      }
      m.kf[id]++;
      face_tets[id].push_back({t, f});
      m.tface[t][f] = id;
    }
  }
  m.n_edges = (int)m.ke.size();
  m.n_faces = (int)m.kf.size();
  for (int f = 0; f < m.n_faces; ++f) {
    if (face_tets[f].size() > 2) throw Failure{E_MESH, "face shared by more than two tets"};
    if (face_tets[f].size() == 2) {
      auto a = face_tets[f][0], b = face_tets[f][1];
      m.tnb[a.first][a.second] = b.first;
      m.tnb[b.first][b.second] = a.first;
    }
  }
  check_links(m);
  int used = 0;
  i64 L = 1;
  bool big = false;
  auto upd = [&](i64 k) {
    if (big) return;
    L = L / gcd64(L, k) * k;
    if (L >= ((i64)1 << 31)) big = true;
  };
  for (int v = 0; v < nv; ++v)
    if (m.kv[v] > 0) {
      ++used;
      upd(m.kv[v]);
    }
  for (int k : m.ke) upd(k);
  for (int k : m.kf) upd(k);
  m.own = force_owner || big;
  m.L = m.own ? 1 : L;
  if (m.own) {  // owner = lowest tet index containing the simplex
    m.ov.assign(nv, -1);
    m.oe.assign(m.n_edges, -1);
    m.of.assign(m.n_faces, -1);
    for (int t = 0; t < nt; ++t) {
      for (int k = 0; k < 4; ++k)
        if (m.ov[m.tv[t][k]] < 0) m.ov[m.tv[t][k]] = t;
      for (int e = 0; e < 6; ++e)
        if (m.oe[m.tedge[t][e]] < 0) m.oe[m.tedge[t][e]] = t;
      for (int f = 0; f < 4; ++f)
        if (m.of[m.tface[t][f]] < 0) m.of[m.tface[t][f]] = t;
    }
  }
  m.n_used_verts = used;
  m.chi = used - m.n_edges + m.n_faces - nt;
  std::vector<int> par(nt);
  std::iota(par.begin(), par.end(), 0);
  for (int t = 0; t < nt; ++t)
    for (int f = 0; f < 4; ++f)
      if (m.tnb[t][f] >= 0) unite(par, t, m.tnb[t][f]);
  int comps = 0;
  for (int t = 0; t < nt; ++t)
    if (find_root(par, t) == t) ++comps;
  m.components = comps;
  return m;
}

struct Sites {
  int n = 0;
  std::vector<i64> X, Y, Z, W;  // centre (grid integers), weight R^2
  std::vector<float> fx, fy, fz, fr;
};

Sites build_sites(int ns, const float* sx, const float* sy, const float* sz, const float* sr) {
  Sites s;
  if (ns <= 0) throw Failure{E_INVALID, "no sites"};
  s.n = ns;
  s.X.resize(ns);
  s.Y.resize(ns);
  s.Z.resize(ns);
  s.W.resize(ns);
  for (int i = 0; i < ns; ++i) {
    i64 r;
    if (!grid_int(sx[i], &s.X[i]) || !grid_int(sy[i], &s.Y[i]) || !grid_int(sz[i], &s.Z[i]) || !grid_int(sr[i], &r))
      throw Failure{E_INVALID, "site value not on the 2^-20 grid or not finite"};
    if (std::llabs(s.X[i]) > (1 << 20) || std::llabs(s.Y[i]) > (1 << 20) || std::llabs(s.Z[i]) > (1 << 20))
      throw Failure{E_INVALID, "site centre outside [-1,1]"};
    if (r < 0 || r > (2 << 20)) throw Failure{E_INVALID, "site radius negative or above 2"};
    s.W[i] = r * r;
  }
  return s;
}

// power distance of grid point (x,y,z) to site j, in units of 2^-40 (exact: |value| < 2^45)
inline i64 pow_dist(const Sites& s, int j, i64 x, i64 y, i64 z) {
  i64 dx = x - s.X[j], dy = y - s.Y[j], dz = z - s.Z[j];
  return dx * dx + dy * dy + dz * dz - s.W[j];
}

// ---------------------------------------------------------------------------------------------------------------
// One piece P_{t,i}: plane list + vertices as plane-index triples (sorted).
// ---------------------------------------------------------------------------------------------------------------
struct Piece {
  std::vector<Plane> planes;
  std::vector<std::array<int, 3>> verts;
};

int shared_planes(const std::array<int, 3>& u, const std::array<int, 3>& w, int out[3]) {
  int c = 0;
  for (int a : u)
    for (int b : w)
      if (a == b) out[c++] = a;
  return c;
}

// Clip the piece of site si by plane q (exact, ties by symbolic perturbation). Returns false when it empties.
bool clip(Piece& P, const Plane& q, int si) {
  int nv = (int)P.verts.size();
  std::vector<int> side(nv);
  bool any_out = false, all_out = true;
  for (int v = 0; v < nv; ++v) {
    const auto& t = P.verts[v];
    int dz = 0;
    int s = side_sos(P.planes[t[0]], P.planes[t[1]], P.planes[t[2]], q, si, &dz);
    if (dz) throw Failure{E_DEGENERATE, "vertex planes without a unique intersection"};
    if (s == 0) throw Failure{E_DEGENERATE, "a perturbed predicate is still zero"};
    side[v] = s;
    if (s < 0) any_out = true;
    else all_out = false;
  }
  if (!any_out) return true;
  if (all_out) {
    P.verts.clear();
    return false;
  }
  int qi = (int)P.planes.size();
  P.planes.push_back(q);
  std::vector<std::array<int, 3>> next;
  for (int v = 0; v < nv; ++v)
    if (side[v] > 0) next.push_back(P.verts[v]);
  for (int u = 0; u < nv; ++u) {
    if (side[u] < 0) continue;
    for (int w = 0; w < nv; ++w) {
      if (side[w] > 0) continue;
      int sh[3];
      if (shared_planes(P.verts[u], P.verts[w], sh) == 2) {
        std::array<int, 3> nvtx = {sh[0], sh[1], qi};
        std::sort(nvtx.begin(), nvtx.end());
        next.push_back(nvtx);
      }
    }
  }
  P.verts.swap(next);
  return true;
}

// ---------------------------------------------------------------------------------------------------------------
// per-piece results
// ---------------------------------------------------------------------------------------------------------------
struct Key {  // assembly key: carrier (dimension, global id) + sorted site set padded with -1
  int8_t dim;
  int32_t id;
  int32_t s[4];
  bool operator<(const Key& o) const {
    if (dim != o.dim) return dim < o.dim;
    if (id != o.id) return id < o.id;
    for (int k = 0; k < 4; ++k)
      if (s[k] != o.s[k]) return s[k] < o.s[k];
    return false;
  }
  bool operator==(const Key& o) const {
    if (dim != o.dim || id != o.id) return false;
    for (int k = 0; k < 4; ++k)
      if (s[k] != o.s[k]) return false;
    return true;
  }
};

struct Elem {  // element: kind 1 cell (i), 2 face (i<j), 3 edge (i<j<k)
  int8_t kind;
  int32_t s[3];
  bool operator<(const Elem& o) const {
    if (kind != o.kind) return kind < o.kind;
    for (int k = 0; k < 3; ++k)
      if (s[k] != o.s[k]) return s[k] < o.s[k];
    return false;
  }
  bool operator==(const Elem& o) const {
    return kind == o.kind && s[0] == o.s[0] && s[1] == o.s[1] && s[2] == o.s[2];
  }
};

struct AsmRec {  // one cell of an element's complex: cdim 0 vertex, 1 edge, 2 face, 3 volume cell
  Elem e;
  int8_t cdim;
  Key k;
  Key a, b;  // endpoints for edges
};

struct Glue {  // element e has a piece in tet t that touches mesh face (t, f); the partner must exist in tnb[t][f]
  Elem e;
  int32_t t;
  int8_t f;
};

struct PieceOut {
  int t, i;
  int nverts, nplanes;
  double vol, m[3];
  i64 chi_cell;
  std::vector<std::pair<int, i64>> face_terms;                 // (j, numerator) for the face on bisector j
  std::vector<std::tuple<int, int, i64>> edge_terms;           // (j, k) j<k, numerator
  std::vector<long double> edge_len;                          // length of each edge_terms segment
  std::vector<std::array<int, 3>> rpv;                        // (j, k, l) sorted
  std::vector<Glue> glue;
};

struct Ctx {
  const Mesh* M;
  const Sites* S;
  bool assemble;
};

Key make_key(const Mesh& M, int t, int i, const Piece& P, const int* pl, int np) {
  // carrier from the tet-face planes among pl[0..np)
  int faces[3], nf = 0;
  int sites[4], ns = 0;
  sites[ns++] = i;
  for (int k = 0; k < np; ++k) {
    const Plane& q = P.planes[pl[k]];
    if (q.kind == 0) faces[nf++] = q.id;
    else sites[ns++] = q.id;
  }
  Key key;
  std::sort(sites, sites + ns);
  for (int k = 0; k < 4; ++k) key.s[k] = k < ns ? sites[k] : -1;
  if (nf == 0) {
    key.dim = 3;
    key.id = t;
  } else if (nf == 1) {
    key.dim = 2;
    key.id = M.tface[t][faces[0]];
  } else if (nf == 2) {
    int vs[2], c = 0;
    for (int v = 0; v < 4; ++v)
      if (v != faces[0] && v != faces[1]) vs[c++] = v;
    key.dim = 1;
    key.id = M.tedge[t][local_edge(vs[0], vs[1])];
  } else {
    int v = 6 - faces[0] - faces[1] - faces[2];
    key.dim = 0;
    key.id = M.tv[t][v];
  }
  return key;
}

// weight numerator nu = L / k(carrier) of an element with the given planes
i64 weight(const Mesh& M, int t, const Piece& P, const int* pl, int np) {
  int faces[3], nf = 0;
  for (int k = 0; k < np; ++k)
    if (P.planes[pl[k]].kind == 0) faces[nf++] = P.planes[pl[k]].id;
  if (nf == 0) return M.L;
  if (nf == 1) {
    const int f = M.tface[t][faces[0]];
    return M.own ? (M.of[f] == t) : M.L / M.kf[f];
  }
  if (nf == 2) {
    int vs[2], c = 0;
    for (int v = 0; v < 4; ++v)
      if (v != faces[0] && v != faces[1]) vs[c++] = v;
    const int e = M.tedge[t][local_edge(vs[0], vs[1])];
    return M.own ? (M.oe[e] == t) : M.L / M.ke[e];
  }
  int v = 6 - faces[0] - faces[1] - faces[2];
  return M.own ? (M.ov[M.tv[t][v]] == t) : M.L / M.kv[M.tv[t][v]];
}

// Everything the oracle derives from one nonempty piece.
void analyse_piece(const Ctx& C, int t, int i, const Piece& P, PieceOut& out, std::vector<AsmRec>* asmrec) {
  const Mesh& M = *C.M;
  const auto& V = P.verts;
  int nv = (int)V.size();
  out.t = t;
  out.i = i;
  out.nverts = nv;
  // edges: pairs of vertices sharing two planes
  struct E2 {
    int u, w, p0, p1;
  };
  std::vector<E2> edges;
  std::vector<int> deg(nv, 0);
  for (int u = 0; u < nv; ++u)
    for (int w = u + 1; w < nv; ++w) {
      int sh[3];
      int c = shared_planes(V[u], V[w], sh);
      if (c == 2) {
        edges.push_back({u, w, sh[0], sh[1]});
        deg[u]++;
        deg[w]++;
      } else if (c == 3) {
        throw Failure{E_DEGENERATE, "repeated vertex"};
      }
    }
  for (int u = 0; u < nv; ++u)
    if (deg[u] != 3) throw Failure{E_DEGENERATE, "piece is not a simple polytope"};
  // faces: planes used by vertices
  std::vector<int> plane_count(P.planes.size(), 0);
  for (const auto& v : V)
    for (int p : v) plane_count[p]++;
  int nfaces = 0;
  for (size_t p = 0; p < P.planes.size(); ++p)
    if (plane_count[p] > 0) {
      if (plane_count[p] < 3) throw Failure{E_DEGENERATE, "face with fewer than 3 vertices"};
      ++nfaces;
    }
  out.nplanes = nfaces;
  if (nv - (int)edges.size() + nfaces != 2) throw Failure{E_DEGENERATE, "piece boundary is not a sphere"};

  // ---- geometry (FP64 / long double): fan of every face from the vertex centroid
  const auto& q = M.tv[t];
  long double O[3] = {(long double)M.X[q[0]], (long double)M.Y[q[0]], (long double)M.Z[q[0]]};
  std::vector<std::array<long double, 3>> X(nv);
  long double apex[3] = {0, 0, 0};
  for (int v = 0; v < nv; ++v) {
    long double y[3];
    point3(P.planes[V[v][0]], P.planes[V[v][1]], P.planes[V[v][2]], y);
    for (int k = 0; k < 3; ++k) {
      X[v][k] = (O[k] + y[k]) / 1048576.0L;
      apex[k] += X[v][k];
    }
  }
  for (int k = 0; k < 3; ++k) apex[k] /= nv;
  long double vol = 0, mom[3] = {0, 0, 0};
  for (size_t p = 0; p < P.planes.size(); ++p) {
    if (plane_count[p] == 0) continue;
    std::vector<int> fv;
    for (int v = 0; v < nv; ++v)
      if (V[v][0] == (int)p || V[v][1] == (int)p || V[v][2] == (int)p) fv.push_back(v);
    // order the face cycle by walking edges that lie in plane p
    std::vector<int> cyc;
    cyc.push_back(fv[0]);
    int prev = -1, cur = fv[0];
    while ((int)cyc.size() < (int)fv.size()) {
      int nxt = -1;
      for (const auto& e : edges) {
        if (e.p0 != (int)p && e.p1 != (int)p) continue;
        int o = e.u == cur ? e.w : (e.w == cur ? e.u : -1);
        if (o >= 0 && o != prev) {
          nxt = o;
          break;
        }
      }
      if (nxt < 0) throw Failure{E_DEGENERATE, "face cycle broken"};
      prev = cur;
      cur = nxt;
      cyc.push_back(cur);
    }
    for (size_t k = 1; k + 1 < cyc.size(); ++k) {
      const auto& a = X[cyc[0]];
      const auto& b = X[cyc[k]];
      const auto& c = X[cyc[k + 1]];
      long double u[3], w[3], z[3];
      for (int d = 0; d < 3; ++d) {
        u[d] = b[d] - a[d];
        w[d] = c[d] - a[d];
        z[d] = apex[d] - a[d];
      }
      long double det = u[0] * (w[1] * z[2] - w[2] * z[1]) - u[1] * (w[0] * z[2] - w[2] * z[0]) +
                        u[2] * (w[0] * z[1] - w[1] * z[0]);
      long double tv = std::fabs(det) / 6.0L;
      vol += tv;
      for (int d = 0; d < 3; ++d) mom[d] += tv * (a[d] + b[d] + c[d] + apex[d]) / 4.0L;
    }
  }
  out.vol = (double)vol;
  for (int d = 0; d < 3; ++d) out.m[d] = (double)mom[d];

  // ---- fractional Euler characteristic contributions (Sec. 4.1.2), numerators over L
  i64 sv = 0, se = 0, sf = 0;
  for (int v = 0; v < nv; ++v) sv += weight(M, t, P, V[v].data(), 3);
  for (const auto& e : edges) {
    int pl[2] = {e.p0, e.p1};
    se += weight(M, t, P, pl, 2);
  }
  for (size_t p = 0; p < P.planes.size(); ++p)
    if (plane_count[p] > 0) {
      int pl[1] = {(int)p};
      sf += weight(M, t, P, pl, 1);
    }
  out.chi_cell = sv - se + sf - M.L;

  // faces on bisectors: RPF_ij piece; edges on two bisectors: RPE_ijk piece; vertices on three bisectors: RPV
  for (size_t p = 0; p < P.planes.size(); ++p) {
    if (plane_count[p] == 0 || P.planes[p].kind != 1) continue;
    int j = P.planes[p].id;
    i64 fvs = 0, fes = 0;
    for (int v = 0; v < nv; ++v)
      if (V[v][0] == (int)p || V[v][1] == (int)p || V[v][2] == (int)p) fvs += weight(M, t, P, V[v].data(), 3);
    for (const auto& e : edges)
      if (e.p0 == (int)p || e.p1 == (int)p) {
        int pl[2] = {e.p0, e.p1};
        fes += weight(M, t, P, pl, 2);
      }
    out.face_terms.push_back({j, fvs - fes + M.L});
  }
  for (const auto& e : edges) {
    const Plane& a = P.planes[e.p0];
    const Plane& b = P.planes[e.p1];
    if (a.kind != 1 || b.kind != 1) continue;
    i64 w = weight(M, t, P, V[e.u].data(), 3) + weight(M, t, P, V[e.w].data(), 3) - M.L;
    int j = std::min(a.id, b.id), k = std::max(a.id, b.id);
    out.edge_terms.push_back({j, k, w});
    long double d2 = 0;
    for (int d = 0; d < 3; ++d) d2 += (X[e.u][d] - X[e.w][d]) * (X[e.u][d] - X[e.w][d]);
    out.edge_len.push_back(std::sqrt(d2));
  }
  for (int v = 0; v < nv; ++v) {
    const Plane& a = P.planes[V[v][0]];
    const Plane& b = P.planes[V[v][1]];
    const Plane& c = P.planes[V[v][2]];
    if (a.kind == 1 && b.kind == 1 && c.kind == 1) {
      std::array<int, 3> s = {a.id, b.id, c.id};
      std::sort(s.begin(), s.end());
      out.rpv.push_back(s);
    }
  }

  // ---- gluing records across mesh faces (Sec. 4.1.1 traversal): the element piece touches local face f
  auto sorted_elem = [](int kind, int a, int b, int c) {
    Elem e;
    e.kind = (int8_t)kind;
    int s[3] = {a, b, c};
    std::sort(s, s + kind);
    for (int k = 0; k < 3; ++k) e.s[k] = k < kind ? s[k] : -1;
    return e;
  };
  for (size_t p = 0; p < P.planes.size(); ++p)
    if (plane_count[p] > 0 && P.planes[p].kind == 0) out.glue.push_back({sorted_elem(1, i, 0, 0), t, (int8_t)P.planes[p].id});
  for (const auto& e : edges) {
    const Plane& a = P.planes[e.p0];
    const Plane& b = P.planes[e.p1];
    if (a.kind + b.kind != 1) continue;  // one face plane + one bisector
    int f = a.kind == 0 ? a.id : b.id;
    int j = a.kind == 1 ? a.id : b.id;
    out.glue.push_back({sorted_elem(2, i, j, 0), t, (int8_t)f});
  }
  for (int v = 0; v < nv; ++v) {
    int f = -1, js[3], nj = 0, nf = 0;
    for (int k = 0; k < 3; ++k) {
      const Plane& a = P.planes[V[v][k]];
      if (a.kind == 0) {
        f = a.id;
        ++nf;
      } else {
        js[nj++] = a.id;
      }
    }
    if (nf == 1 && nj == 2) out.glue.push_back({sorted_elem(3, i, js[0], js[1]), t, (int8_t)f});
  }

  // ---- explicit assembly records (P7 / skeleton beta0)
  if (!asmrec) return;
  auto push = [&](const Elem& el, int cdim, const Key& k, const Key* a, const Key* b) {
    AsmRec r;
    r.e = el;
    r.cdim = (int8_t)cdim;
    r.k = k;
    if (a) r.a = *a;
    else std::memset(&r.a, 0, sizeof(Key));
    if (b) r.b = *b;
    else std::memset(&r.b, 0, sizeof(Key));
    asmrec->push_back(r);
  };
  std::vector<Key> vkey(nv);
  for (int v = 0; v < nv; ++v) vkey[v] = make_key(M, t, i, P, V[v].data(), 3);
  Elem cell = sorted_elem(1, i, 0, 0);
  for (int v = 0; v < nv; ++v) push(cell, 0, vkey[v], nullptr, nullptr);
  for (const auto& e : edges) {
    int pl[2] = {e.p0, e.p1};
    push(cell, 1, make_key(M, t, i, P, pl, 2), &vkey[e.u], &vkey[e.w]);
  }
  for (size_t p = 0; p < P.planes.size(); ++p)
    if (plane_count[p] > 0) {
      int pl[1] = {(int)p};
      push(cell, 2, make_key(M, t, i, P, pl, 1), nullptr, nullptr);
    }
  {
    Key k;
    k.dim = 3;
    k.id = t;
    k.s[0] = i;
    k.s[1] = k.s[2] = k.s[3] = -1;
    push(cell, 3, k, nullptr, nullptr);
  }
  // faces from the min side only; edges from the min side only
  for (size_t p = 0; p < P.planes.size(); ++p) {
    if (plane_count[p] == 0 || P.planes[p].kind != 1) continue;
    int j = P.planes[p].id;
    if (j < i) continue;
    Elem fe = sorted_elem(2, i, j, 0);
    for (int v = 0; v < nv; ++v)
      if (V[v][0] == (int)p || V[v][1] == (int)p || V[v][2] == (int)p) push(fe, 0, vkey[v], nullptr, nullptr);
    for (const auto& e : edges)
      if (e.p0 == (int)p || e.p1 == (int)p) {
        int pl[2] = {e.p0, e.p1};
        push(fe, 1, make_key(M, t, i, P, pl, 2), &vkey[e.u], &vkey[e.w]);
      }
    int pl[1] = {(int)p};
    push(fe, 2, make_key(M, t, i, P, pl, 1), nullptr, nullptr);
  }
  for (const auto& e : edges) {
    const Plane& a = P.planes[e.p0];
    const Plane& b = P.planes[e.p1];
    if (a.kind != 1 || b.kind != 1) continue;
    if (a.id < i || b.id < i) continue;
    Elem ee = sorted_elem(3, i, a.id, b.id);
    push(ee, 0, vkey[e.u], nullptr, nullptr);
    push(ee, 0, vkey[e.w], nullptr, nullptr);
    int pl[2] = {e.p0, e.p1};
    push(ee, 1, make_key(M, t, i, P, pl, 2), &vkey[e.u], &vkey[e.w]);
  }
}

Plane face_plane(const Mesh& M, int t, int f) {
  const auto& q = M.tv[t];
  i64 ox = M.X[q[0]], oy = M.Y[q[0]], oz = M.Z[q[0]];
  int o[3], c = 0;
  for (int k = 0; k < 4; ++k)
    if (k != f) o[c++] = k;
  auto P = [&](int k, i128* p) {
    p[0] = M.X[q[k]] - ox;
    p[1] = M.Y[q[k]] - oy;
    p[2] = M.Z[q[k]] - oz;
  };
  i128 a[3], b[3], cc[3], v[3];
  P(o[0], a);
  P(o[1], b);
  P(o[2], cc);
  P(f, v);
  i128 u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  i128 w[3] = {cc[0] - a[0], cc[1] - a[1], cc[2] - a[2]};
  Plane pl;
  pl.n[0] = u[1] * w[2] - u[2] * w[1];
  pl.n[1] = u[2] * w[0] - u[0] * w[2];
  pl.n[2] = u[0] * w[1] - u[1] * w[0];
  i128 s = pl.n[0] * (v[0] - a[0]) + pl.n[1] * (v[1] - a[1]) + pl.n[2] * (v[2] - a[2]);
  if (s < 0)
    for (int k = 0; k < 3; ++k) pl.n[k] = -pl.n[k];
  pl.d = -(pl.n[0] * a[0] + pl.n[1] * a[1] + pl.n[2] * a[2]);
  pl.kind = 0;
  pl.id = f;
  return pl;
}

// The brute-force clip of one tet against every site (Sec. 5.2 Tet-Cell, all sites as neighbours).
void process_tet(const Ctx& C, int t, std::vector<PieceOut>& outs, std::vector<AsmRec>* asmrec, i64* attempted) {
  const Mesh& M = *C.M;
  const Sites& S = *C.S;
  const auto& q = M.tv[t];
  i64 ox = M.X[q[0]], oy = M.Y[q[0]], oz = M.Z[q[0]];
  int n = S.n;
  // power distance of every site at the 4 tet vertices (exact) and at the centroid (for the visiting order)
  std::vector<std::array<i64, 4>> Dv(n);
  std::vector<std::pair<double, int>> order(n);
  double cx = 0, cy = 0, cz = 0;
  for (int k = 0; k < 4; ++k) {
    cx += M.X[q[k]] * 0.25;
    cy += M.Y[q[k]] * 0.25;
    cz += M.Z[q[k]] * 0.25;
  }
  for (int j = 0; j < n; ++j) {
    for (int k = 0; k < 4; ++k) Dv[j][k] = pow_dist(S, j, M.X[q[k]], M.Y[q[k]], M.Z[q[k]]);
    double dx = cx - S.X[j], dy = cy - S.Y[j], dz = cz - S.Z[j];
    order[j] = {dx * dx + dy * dy + dz * dz - (double)S.W[j], j};
  }
  std::sort(order.begin(), order.end());
  Plane faces[4];
  for (int f = 0; f < 4; ++f) faces[f] = face_plane(M, t, f);
  // P_{t,i} starts as the tet itself: its four face planes, and vertex v as the meet of the three faces other than
  // face v. It is set up when the first plane cuts the tet (a plane that keeps or removes the whole tet is decided
  // at the four vertices alone); the storage is reused from site to site.
  Piece P;
  auto start_as_tet = [&]() {
    P.planes.assign(faces, faces + 4);
    P.verts.clear();
    for (int v = 0; v < 4; ++v) {
      std::array<int, 3> tri;
      int c = 0;
      for (int f = 0; f < 4; ++f)
        if (f != v) tri[c++] = f;
      P.verts.push_back(tri);
    }
  };
  for (int oi = 0; oi < n; ++oi) {
    int i = order[oi].second;
    ++*attempted;
    bool started = false;
    bool alive = true;
    for (int oj = 0; oj < n && alive; ++oj) {
      int j = order[oj].second;
      if (j == i) continue;
      // h_ij = d_j - d_i is affine; its values at the tet vertices are exact
      bool all_pos = true, all_neg = true;
      for (int k = 0; k < 4; ++k) {
        i64 h = Dv[j][k] - Dv[i][k];
        if (h <= 0) all_pos = false;
        if (h >= 0) all_neg = false;
      }
      if (all_pos) continue;  // t lies inside H_ij, so the clip is a no-op
      if (all_neg) {          // t lies outside H_ij, so the piece is empty
        alive = false;
        break;
      }
      Plane h;
      h.n[0] = 2 * (i128)(S.X[i] - S.X[j]);
      h.n[1] = 2 * (i128)(S.Y[i] - S.Y[j]);
      h.n[2] = 2 * (i128)(S.Z[i] - S.Z[j]);
      h.d = (i128)pow_dist(S, j, ox, oy, oz) - (i128)pow_dist(S, i, ox, oy, oz);
      h.kind = 1;
      h.id = j;
      if (!started) {
        start_as_tet();
        started = true;
      }
      alive = clip(P, h, i);
    }
    if (!alive) continue;
    if (!started) start_as_tet();  // no plane cuts the tet: the piece is the whole tet
    if (P.verts.empty()) continue;
    PieceOut po;
    analyse_piece(C, t, i, P, po, asmrec);
    outs.push_back(std::move(po));
  }
}

static void set_msg(char* dst, const std::string& s) {
  std::snprintf(dst, 256, "%s", s.c_str());
}

template <class T>
static T* dup(const std::vector<T>& v) {
  T* p = (T*)std::malloc(sizeof(T) * (v.size() ? v.size() : 1));
  if (!v.empty()) std::memcpy(p, v.data(), sizeof(T) * v.size());
  return p;
}

static void run_tets(const Ctx& C, const std::vector<int>& tets, int nthreads, std::vector<PieceOut>& all,
                     std::vector<AsmRec>* asmall, i64* attempted, Failure* fail) {
  if (nthreads <= 0) nthreads = (int)std::thread::hardware_concurrency();
  if (nthreads <= 0) nthreads = 1;
  std::atomic<size_t> next(0);
  std::vector<std::vector<PieceOut>> per(nthreads);
  std::vector<std::vector<AsmRec>> pera(nthreads);
  std::vector<i64> att(nthreads, 0);
  std::mutex mu;
  bool failed = false;
  auto work = [&](int w) {
    try {
      while (true) {
        size_t k = next.fetch_add(16);
        if (k >= tets.size()) break;
        size_t e = std::min(tets.size(), k + 16);
        for (size_t x = k; x < e; ++x) process_tet(C, tets[x], per[w], asmall ? &pera[w] : nullptr, &att[w]);
        if (failed) break;
      }
    } catch (const Failure& f) {
      std::lock_guard<std::mutex> g(mu);
      if (!failed) *fail = f;
      failed = true;
    } catch (const std::bad_alloc&) {
      std::lock_guard<std::mutex> g(mu);
      if (!failed) *fail = Failure{E_NOMEM, "out of host memory"};
      failed = true;
    }
  };
  std::vector<std::thread> th;
  for (int w = 0; w < nthreads; ++w) th.emplace_back(work, w);
  for (auto& x : th) x.join();
  if (failed) return;
  for (int w = 0; w < nthreads; ++w) {
    for (auto& p : per[w]) all.push_back(std::move(p));
    if (asmall) asmall->insert(asmall->end(), pera[w].begin(), pera[w].end());
    *attempted += att[w];
  }
  std::sort(all.begin(), all.end(), [](const PieceOut& a, const PieceOut& b) {
    return a.t != b.t ? a.t < b.t : a.i < b.i;
  });
}

}  // namespace

// ===============================================================================================================
// C ABI for the Python test driver
// ===============================================================================================================
extern "C" {

typedef struct oracle_result {
  int32_t status;
  char msg[256];
  int64_t L;
  int32_t mesh_chi;
  int32_t mesh_components;
  int32_t n_sites;
  int64_t n_pairs;      // nonempty pieces P_{t,i}
  int64_t n_attempted;  // (t,i) pairs visited
  int32_t consistent;   // 1 if every internal cross-check passed
  char report[512];
  // cells [n_sites]
  int32_t* cell_chi;
  int32_t* cell_chi_asm;
  int32_t* cell_beta0;
  int32_t* cell_beta0_skel;
  double* cell_vol;
  double* cell_cen;  // 3 n
  int64_t* cell_npieces;
  // faces
  int64_t n_faces;
  int32_t* face_keys;  // 2 per face, ascending
  int32_t* face_chi;
  int32_t* face_chi_asm;
  int32_t* face_beta0;
  int32_t* face_beta0_skel;
  // edges
  int64_t n_edges;
  int32_t* edge_keys;  // 3 per edge
  int32_t* edge_chi;
  int32_t* edge_chi_asm;
  int32_t* edge_beta0;
  int32_t* edge_beta0_skel;
  double* edge_length;  // summed segment lengths of the RPE's pieces (Sec. 5.3, importance of the dual triangle)
  // RPV quads
  int64_t n_rpv;
  int32_t* rpv_keys;  // 4 per quad
  // per-piece statistics
  int32_t max_piece_verts;
  int32_t max_piece_faces;
  // the connected component of every cell piece: (t, i, label), labels equal iff the pieces of cell i are glued
  // into one component (Sec. 4.1.1); ordered by (i, t)
  int64_t n_cell_pieces;
  int32_t* cell_piece;  // 3 per piece
} oracle_result;

typedef struct oracle_piece {  // one nonempty piece, for sampled comparisons
  int32_t t, i;
  int32_t nverts, nfaces;
  double vol, m[3];
  int64_t chi_cell;  // numerator over L
  int32_t n_face_terms, n_edge_terms, n_rpv, n_glue;
  int32_t off_face, off_edge, off_rpv, off_glue;
} oracle_piece;

typedef struct oracle_pieces {
  int32_t status;
  char msg[256];
  int64_t L;
  int64_t n;
  oracle_piece* pieces;
  int32_t* face_terms;  // (j, lo32(num), hi32(num)) triples
  int32_t* edge_terms;  // (j, k, lo32, hi32)
  int32_t* rpv;         // (j, k, l)
  int32_t* glue;        // (kind, s0, s1, s2, f)
} oracle_pieces;

void oracle_free(oracle_result* r);
void oracle_pieces_free(oracle_pieces* r);

int oracle_rpd(int32_t nv, const float* vx, const float* vy, const float* vz, int32_t nt, const int32_t* tv,
               int32_t ns, const float* sx, const float* sy, const float* sz, const float* sr, int32_t nthreads,
               int32_t assemble, int32_t owner_weights, oracle_result** out) {
  oracle_result* R = (oracle_result*)std::calloc(1, sizeof(oracle_result));
  *out = R;
  try {
    Mesh M = build_mesh(nv, vx, vy, vz, nt, tv, owner_weights != 0);
    Sites S = build_sites(ns, sx, sy, sz, sr);
    R->L = M.L;
    R->mesh_chi = M.chi;
    R->mesh_components = M.components;
    R->n_sites = ns;
    Ctx C{&M, &S, assemble != 0};
    std::vector<int> tets(nt);
    std::iota(tets.begin(), tets.end(), 0);
    std::vector<PieceOut> pcs;
    std::vector<AsmRec> asmr;
    i64 attempted = 0;
    Failure fail{OK, ""};
    run_tets(C, tets, nthreads, pcs, assemble ? &asmr : nullptr, &attempted, &fail);
    if (fail.code != OK) throw fail;
    R->n_pairs = (int64_t)pcs.size();
    R->n_attempted = attempted;
    std::string report;
    bool consistent = true;
    auto flag = [&](const std::string& s) {
      if (consistent) report = s;
      consistent = false;
    };

    // ---- cells
    std::vector<i64> cnum(ns, 0);
    std::vector<long double> vol(ns, 0), mom(3 * ns, 0);
    std::vector<int64_t> npieces(ns, 0);
    int maxv = 0, maxf = 0;
    for (const auto& p : pcs) {
      cnum[p.i] += p.chi_cell;
      vol[p.i] += p.vol;
      for (int d = 0; d < 3; ++d) mom[3 * p.i + d] += p.m[d];
      npieces[p.i]++;
      maxv = std::max(maxv, p.nverts);
      maxf = std::max(maxf, p.nplanes);
    }
    R->max_piece_verts = maxv;
    R->max_piece_faces = maxf;
    std::vector<int32_t> cchi(ns);
    std::vector<double> cvol(ns), ccen(3 * ns);
    for (int i = 0; i < ns; ++i) {
      if (cnum[i] % M.L != 0) flag("cell fractional chi not an integer");
      cchi[i] = (int32_t)(cnum[i] / M.L);
      cvol[i] = (double)vol[i];
      for (int d = 0; d < 3; ++d)
        ccen[3 * i + d] = npieces[i] ? (double)(mom[3 * i + d] / vol[i]) : std::nan("");
    }
    // ---- faces, from every side: num[side 0 = min site, side 1 = max site]
    std::map<std::pair<int, int>, std::array<i64, 2>> fnum;
    std::map<std::pair<int, int>, std::array<int, 2>> fcount;
    std::map<std::array<int, 3>, std::array<i64, 3>> enumr;
    std::map<std::array<int, 3>, std::array<int, 3>> ecount;
    std::map<std::array<int, 3>, std::array<long double, 3>> elen;
    std::map<std::array<int, 4>, int> rpvc;
    for (const auto& p : pcs) {
      for (const auto& ft : p.face_terms) {
        auto key = std::make_pair(std::min(p.i, ft.first), std::max(p.i, ft.first));
        int side = p.i == key.first ? 0 : 1;
        auto& a = fnum[key];
        a[side] += ft.second;
        fcount[key][side]++;
      }
      for (const auto& et : p.edge_terms) {
        std::array<int, 3> key = {p.i, std::get<0>(et), std::get<1>(et)};
        std::sort(key.begin(), key.end());
        int side = p.i == key[0] ? 0 : (p.i == key[1] ? 1 : 2);
        enumr[key][side] += std::get<2>(et);
        ecount[key][side]++;
      }
      for (size_t q = 0; q < p.edge_terms.size(); ++q) {
        const auto& et = p.edge_terms[q];
        std::array<int, 3> key = {p.i, std::get<0>(et), std::get<1>(et)};
        std::sort(key.begin(), key.end());
        int side = p.i == key[0] ? 0 : (p.i == key[1] ? 1 : 2);
        elen[key][side] += p.edge_len[q];
      }
      for (const auto& r : p.rpv) {
        std::array<int, 4> key = {p.i, r[0], r[1], r[2]};
        std::sort(key.begin(), key.end());
        rpvc[key]++;
      }
    }
    std::vector<int32_t> fkeys, fchi;
    std::map<std::pair<int, int>, int> fidx;
    for (const auto& kv : fnum) {
      if (kv.second[0] != kv.second[1]) flag("face fractional chi differs between its two sides");
      if (fcount[kv.first][0] != fcount[kv.first][1]) flag("face piece count differs between sides");
      if (kv.second[0] % M.L != 0) flag("face fractional chi not an integer");
      fidx[kv.first] = (int)fkeys.size() / 2;
      fkeys.push_back(kv.first.first);
      fkeys.push_back(kv.first.second);
      fchi.push_back((int32_t)(kv.second[0] / M.L));
    }
    std::vector<int32_t> ekeys, echi;
    std::vector<double> elength;
    std::map<std::array<int, 3>, int> eidx;
    for (const auto& kv : enumr) {
      if (kv.second[0] != kv.second[1] || kv.second[0] != kv.second[2])
        flag("edge fractional chi differs between its sides");
      auto c = ecount[kv.first];
      if (c[0] != c[1] || c[0] != c[2]) flag("edge piece count differs between sides");
      if (kv.second[0] % M.L != 0) flag("edge fractional chi not an integer");
      eidx[kv.first] = (int)ekeys.size() / 3;
      for (int k = 0; k < 3; ++k) ekeys.push_back(kv.first[k]);
      echi.push_back((int32_t)(kv.second[0] / M.L));
      // the same segments seen from the three cells: lengths agree up to rounding
      const auto& l3 = elen[kv.first];
      for (int sd = 1; sd < 3; ++sd)
        if (std::fabs(l3[sd] - l3[0]) > 1e-12L * (1 + l3[0])) flag("edge length differs between its sides");
      elength.push_back((double)l3[0]);
    }
    std::vector<int32_t> rkeys;
    for (const auto& kv : rpvc) {
      if (kv.second != 4) flag("RPV not seen from exactly four cells");
      for (int k = 0; k < 4; ++k) rkeys.push_back(kv.first[k]);
    }
    // ---- beta0 by union-find over glued element pieces
    std::map<std::pair<Elem, int>, int> node;  // (element, tet) -> node id
    std::vector<std::tuple<Elem, int, int>> glue_list;  // element, t, f
    for (const auto& p : pcs) {
      // register element pieces from their canonical (min-site) side only
      Elem ce;
      ce.kind = 1;
      ce.s[0] = p.i;
      ce.s[1] = ce.s[2] = -1;
      node.emplace(std::make_pair(ce, p.t), (int)node.size());
      for (const auto& ft : p.face_terms)
        if (ft.first > p.i) {
          Elem e;
          e.kind = 2;
          e.s[0] = p.i;
          e.s[1] = ft.first;
          e.s[2] = -1;
          node.emplace(std::make_pair(e, p.t), (int)node.size());
        }
      for (const auto& et : p.edge_terms)
        if (std::get<0>(et) > p.i) {
          Elem e;
          e.kind = 3;
          e.s[0] = p.i;
          e.s[1] = std::get<0>(et);
          e.s[2] = std::get<1>(et);
          node.emplace(std::make_pair(e, p.t), (int)node.size());
        }
      for (const auto& g : p.glue)
        if (g.e.s[0] == p.i) glue_list.push_back({g.e, g.t, g.f});
    }
    std::vector<int> par(node.size());
    std::iota(par.begin(), par.end(), 0);
    std::map<std::tuple<Elem, int, int>, int> glue_seen;  // (element, t, neighbour t') seen
    for (const auto& g : glue_list) {
      const Elem& e = std::get<0>(g);
      int t = std::get<1>(g), f = std::get<2>(g);
      int t2 = M.tnb[t][f];
      if (t2 < 0) continue;
      auto a = node.find({e, t});
      auto b = node.find({e, t2});
      if (a == node.end() || b == node.end()) {
        flag("gluing record without a partner piece across the mesh face");
        continue;
      }
      unite(par, a->second, b->second);
      glue_seen[std::make_tuple(e, std::min(t, t2), std::max(t, t2))]++;
    }
    for (const auto& kv : glue_seen)
      if (kv.second != 2) flag("gluing record not symmetric across a mesh face");
    std::vector<int32_t> cb0(ns, 0), fb0(fkeys.size() / 2, 0), eb0(ekeys.size() / 3, 0);
    std::vector<int32_t> cell_piece;  // (t, i, root) of every cell piece, in (i, t) order (the map's order)
    for (const auto& kv : node)
      if (kv.first.first.kind == 1) {
        cell_piece.push_back(kv.first.second);
        cell_piece.push_back(kv.first.first.s[0]);
        cell_piece.push_back(find_root(par, kv.second));
      }
    for (const auto& kv : node) {
      if (find_root(par, kv.second) != kv.second) continue;
      const Elem& e = kv.first.first;
      if (e.kind == 1) cb0[e.s[0]]++;
      else if (e.kind == 2) fb0[fidx[{e.s[0], e.s[1]}]]++;
      else eb0[eidx[{e.s[0], e.s[1], e.s[2]}]]++;
    }
    // ---- explicit assembly
    std::vector<int32_t> cchi_a(ns, 0), fchi_a(fb0.size(), 0), echi_a(eb0.size(), 0);
    std::vector<int32_t> cb0s(ns, 0), fb0s(fb0.size(), 0), eb0s(eb0.size(), 0);
    if (assemble) {
      auto lessrec = [](const AsmRec& x, const AsmRec& y) {
        if (!(x.e == y.e)) return x.e < y.e;
        if (x.cdim != y.cdim) return x.cdim < y.cdim;
        return x.k < y.k;
      };
      std::sort(asmr.begin(), asmr.end(), lessrec);
      auto elem_chi = [&](const Elem& e) -> int32_t* {
        if (e.kind == 1) return &cchi_a[e.s[0]];
        if (e.kind == 2) return &fchi_a[fidx[{e.s[0], e.s[1]}]];
        return &echi_a[eidx[{e.s[0], e.s[1], e.s[2]}]];
      };
      auto elem_b0 = [&](const Elem& e) -> int32_t* {
        if (e.kind == 1) return &cb0s[e.s[0]];
        if (e.kind == 2) return &fb0s[fidx[{e.s[0], e.s[1]}]];
        return &eb0s[eidx[{e.s[0], e.s[1], e.s[2]}]];
      };
      size_t a = 0;
      while (a < asmr.size()) {
        size_t b = a;
        while (b < asmr.size() && asmr[b].e == asmr[a].e) ++b;
        // distinct cells per dimension; vertices indexed for the skeleton union-find
        int counts[4] = {0, 0, 0, 0};
        std::vector<Key> vk;
        std::vector<std::pair<Key, Key>> ek;
        for (size_t x = a; x < b; ++x) {
          if (x > a && asmr[x].cdim == asmr[x - 1].cdim && asmr[x].k == asmr[x - 1].k) continue;
          counts[asmr[x].cdim]++;
          if (asmr[x].cdim == 0) vk.push_back(asmr[x].k);
          if (asmr[x].cdim == 1) ek.push_back({asmr[x].a, asmr[x].b});
        }
        *elem_chi(asmr[a].e) = counts[0] - counts[1] + counts[2] - counts[3];
        std::vector<int> up(vk.size());
        std::iota(up.begin(), up.end(), 0);
        auto vid = [&](const Key& k) {
          return (int)(std::lower_bound(vk.begin(), vk.end(), k) - vk.begin());
        };
        for (const auto& e : ek) unite(up, vid(e.first), vid(e.second));
        int comps = 0;
        for (size_t x = 0; x < up.size(); ++x)
          if (find_root(up, (int)x) == (int)x) ++comps;
        *elem_b0(asmr[a].e) = comps;
        a = b;
      }
      for (int i = 0; i < ns; ++i) {
        if (cchi_a[i] != cchi[i]) flag("cell: fractional chi differs from assembled chi");
        if (cb0s[i] != cb0[i]) flag("cell: glued beta0 differs from skeleton beta0");
      }
      for (size_t k = 0; k < fchi.size(); ++k) {
        if (fchi_a[k] != fchi[k]) flag("face: fractional chi differs from assembled chi");
        if (fb0s[k] != fb0[k]) flag("face: glued beta0 differs from skeleton beta0");
      }
      for (size_t k = 0; k < echi.size(); ++k) {
        if (echi_a[k] != echi[k]) flag("edge: fractional chi differs from assembled chi");
        if (eb0s[k] != eb0[k]) flag("edge: glued beta0 differs from skeleton beta0");
      }
    } else {
      cchi_a = cchi;
      fchi_a = fchi;
      echi_a = echi;
      cb0s = cb0;
      fb0s = fb0;
      eb0s = eb0;
    }
    R->consistent = consistent ? 1 : 0;
    set_msg(R->report, consistent ? "ok" : report);
    R->cell_chi = dup(cchi);
    R->cell_chi_asm = dup(cchi_a);
    R->cell_beta0 = dup(cb0);
    R->cell_beta0_skel = dup(cb0s);
    R->cell_vol = dup(cvol);
    R->cell_cen = dup(ccen);
    R->cell_npieces = dup(npieces);
    R->n_faces = (int64_t)fchi.size();
    R->face_keys = dup(fkeys);
    R->face_chi = dup(fchi);
    R->face_chi_asm = dup(fchi_a);
    R->face_beta0 = dup(fb0);
    R->face_beta0_skel = dup(fb0s);
    R->n_edges = (int64_t)echi.size();
    R->edge_keys = dup(ekeys);
    R->edge_chi = dup(echi);
    R->edge_chi_asm = dup(echi_a);
    R->edge_beta0 = dup(eb0);
    R->edge_beta0_skel = dup(eb0s);
    R->edge_length = dup(elength);
    R->n_rpv = (int64_t)rkeys.size() / 4;
    R->rpv_keys = dup(rkeys);
    R->n_cell_pieces = (int64_t)cell_piece.size() / 3;
    R->cell_piece = dup(cell_piece);
    R->status = OK;
    set_msg(R->msg, "ok");
  } catch (const Failure& f) {
    R->status = f.code;
    set_msg(R->msg, f.msg);
  } catch (const std::bad_alloc&) {
    R->status = E_NOMEM;
    set_msg(R->msg, "out of host memory");
  }
  return R->status;
}

// Per-piece results for a chosen list of tets (each tet still clipped against ALL sites).
int oracle_tet_pieces(int32_t nv, const float* vx, const float* vy, const float* vz, int32_t nt, const int32_t* tv,
                      int32_t ns, const float* sx, const float* sy, const float* sz, const float* sr,
                      int32_t n_sel, const int32_t* sel, int32_t nthreads, int32_t owner_weights,
                      oracle_pieces** out) {
  oracle_pieces* R = (oracle_pieces*)std::calloc(1, sizeof(oracle_pieces));
  *out = R;
  try {
    Mesh M = build_mesh(nv, vx, vy, vz, nt, tv, owner_weights != 0);
    Sites S = build_sites(ns, sx, sy, sz, sr);
    Ctx C{&M, &S, false};
    std::vector<int> tets;
    for (int k = 0; k < n_sel; ++k) {
      if (sel[k] < 0 || sel[k] >= nt) throw Failure{E_INVALID, "selected tet out of range"};
      tets.push_back(sel[k]);
    }
    std::vector<PieceOut> pcs;
    i64 attempted = 0;
    Failure fail{OK, ""};
    run_tets(C, tets, nthreads, pcs, nullptr, &attempted, &fail);
    if (fail.code != OK) throw fail;
    std::vector<oracle_piece> P;
    std::vector<int32_t> ft, et, rv, gl;
    for (const auto& p : pcs) {
      oracle_piece o;
      o.t = p.t;
      o.i = p.i;
      o.nverts = p.nverts;
      o.nfaces = p.nplanes;
      o.vol = p.vol;
      for (int d = 0; d < 3; ++d) o.m[d] = p.m[d];
      o.chi_cell = p.chi_cell;
      o.off_face = (int32_t)ft.size() / 3;
      o.n_face_terms = (int32_t)p.face_terms.size();
      for (const auto& x : p.face_terms) {
        ft.push_back(x.first);
        ft.push_back((int32_t)(uint32_t)(uint64_t)x.second);
        ft.push_back((int32_t)(uint32_t)((uint64_t)x.second >> 32));
      }
      o.off_edge = (int32_t)et.size() / 4;
      o.n_edge_terms = (int32_t)p.edge_terms.size();
      for (const auto& x : p.edge_terms) {
        et.push_back(std::get<0>(x));
        et.push_back(std::get<1>(x));
        i64 v = std::get<2>(x);
        et.push_back((int32_t)(uint32_t)(uint64_t)v);
        et.push_back((int32_t)(uint32_t)((uint64_t)v >> 32));
      }
      o.off_rpv = (int32_t)rv.size() / 3;
      o.n_rpv = (int32_t)p.rpv.size();
      for (const auto& x : p.rpv)
        for (int k = 0; k < 3; ++k) rv.push_back(x[k]);
      o.off_glue = (int32_t)gl.size() / 5;
      o.n_glue = (int32_t)p.glue.size();
      for (const auto& g : p.glue) {
        gl.push_back(g.e.kind);
        for (int k = 0; k < 3; ++k) gl.push_back(g.e.s[k]);
        gl.push_back(g.f);
      }
      P.push_back(o);
    }
    R->L = M.L;
    R->n = (int64_t)P.size();
    R->pieces = dup(P);
    R->face_terms = dup(ft);
    R->edge_terms = dup(et);
    R->rpv = dup(rv);
    R->glue = dup(gl);
    R->status = OK;
    set_msg(R->msg, "ok");
  } catch (const Failure& f) {
    R->status = f.code;
    set_msg(R->msg, f.msg);
  } catch (const std::bad_alloc&) {
    R->status = E_NOMEM;
    set_msg(R->msg, "out of host memory");
  }
  return R->status;
}

// Exact side test exposed for the predicate pins: planes as (nx, ny, nz, d) rows of 128-bit integers given as
// (lo, hi) 64-bit halves.  Returns the sign of plane 3 at the meet of planes 0, 1, 2 (or 2 if they do not meet
// in a single point).
int oracle_side_exact(const int64_t* rows_lohi) {
  Plane p[4];
  for (int r = 0; r < 4; ++r) {
    i128 c[4];
    for (int k = 0; k < 4; ++k) {
      uint64_t lo = (uint64_t)rows_lohi[8 * r + 2 * k];
      uint64_t hi = (uint64_t)rows_lohi[8 * r + 2 * k + 1];
      c[k] = (i128)(((u128)hi << 64) | lo);
    }
    p[r].n[0] = c[0];
    p[r].n[1] = c[1];
    p[r].n[2] = c[2];
    p[r].d = c[3];
    p[r].kind = 1;
    p[r].id = r;
  }
  int dz = 0;
  int s = side_exact(p[0], p[1], p[2], p[3], &dz);
  return dz ? 2 : s;
}

void oracle_free(oracle_result* r) {
  if (!r) return;
  void* ptrs[] = {r->cell_chi,   r->cell_chi_asm,    r->cell_beta0,   r->cell_beta0_skel, r->cell_vol,
                  r->cell_cen,   r->cell_npieces,    r->face_keys,    r->face_chi,        r->face_chi_asm,
                  r->face_beta0, r->face_beta0_skel, r->edge_keys,    r->edge_chi,        r->edge_chi_asm,
                  r->edge_beta0, r->edge_beta0_skel, r->edge_length, r->rpv_keys, r->cell_piece};
  for (void* p : ptrs) std::free(p);
  std::free(r);
}

void oracle_pieces_free(oracle_pieces* r) {
  if (!r) return;
  std::free(r->pieces);
  std::free(r->face_terms);
  std::free(r->edge_terms);
  std::free(r->rpv);
  std::free(r->glue);
  std::free(r);
}

}  // extern "C"
