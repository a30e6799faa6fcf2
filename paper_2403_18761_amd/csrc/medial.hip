// Dual medial mesh of an RPD and its geometry-guided thinning (Sec. 3.2 duality, Sec. 5.3 thinning).
//
// Thinning is a greedy sequence of simple-pair removals on a small simplicial complex (one entry per RPV, RPE and
// RPF), each step depending on the previous one; it runs on the host over the arrays the device produced (element
// keys and the importance alpha of every medial triangle), not on the clipping path.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <queue>
#include <tuple>
#include <vector>

#include "rpd.h"
#include "rpd_host.h"

namespace rpd {
namespace {

template <int K>
bool lex_less(const int32_t* a, const int32_t* b) {
  for (int c = 0; c < K; ++c)
    if (a[c] != b[c]) return a[c] < b[c];
  return false;
}

// index of key in a sorted array of K-tuples, or -1
template <int K>
long long find_key(const int32_t* arr, long long n, const int32_t* key) {
  long long lo = 0, hi = n;
  while (lo < hi) {
    long long mid = (lo + hi) / 2;
    if (lex_less<K>(arr + K * mid, key)) lo = mid + 1;
    else hi = mid;
  }
  if (lo < n && !lex_less<K>(key, arr + K * lo)) return lo;
  return -1;
}

template <int K>
void check_simplices(const int32_t* arr, long long n, int nv, const char* what) {
  if (n < 0 || (n > 0 && !arr)) throw Failure{RPD_E_INVALID, std::string(what) + ": bad count or null array"};
  for (long long q = 0; q < n; ++q) {
    const int32_t* s = arr + K * q;
    for (int c = 0; c < K; ++c) {
      if (s[c] < 0 || s[c] >= nv) throw Failure{RPD_E_INVALID, std::string(what) + ": vertex id out of range"};
      if (c && s[c - 1] >= s[c]) throw Failure{RPD_E_INVALID, std::string(what) + ": ids not strictly ascending"};
    }
    if (q && !lex_less<K>(arr + K * (q - 1), s))
      throw Failure{RPD_E_INVALID, std::string(what) + ": not sorted strictly ascending"};
  }
}

struct Csr {  // incidence lists: items of owner o are idx[off[o] .. off[o + 1])
  std::vector<long long> off, idx;
  void build(long long n_owner, const std::vector<std::pair<long long, long long>>& pairs) {
    off.assign(n_owner + 1, 0);
    for (const auto& p : pairs) off[p.first + 1]++;
    for (long long o = 0; o < n_owner; ++o) off[o + 1] += off[o];
    idx.resize(pairs.size());
    std::vector<long long> cur(off.begin(), off.end() - 1);
    for (const auto& p : pairs) idx[cur[p.first]++] = p.second;
  }
};

}  // namespace

void thin(int nv, long long ne, const int32_t* edges, long long nf, const int32_t* tris, const double* alpha,
          long long nt, const int32_t* tets, double sigma, uint8_t* keep_e, uint8_t* keep_f, uint8_t* keep_t) {
  if (nv < 0) throw Failure{RPD_E_INVALID, "n_vertices < 0"};
  check_simplices<2>(edges, ne, nv, "edges");
  check_simplices<3>(tris, nf, nv, "triangles");
  check_simplices<4>(tets, nt, nv, "tets");
  if (nf > 0 && !alpha) throw Failure{RPD_E_INVALID, "alpha is null"};
  for (long long f = 0; f < nf; ++f)
    if (std::isnan(alpha[f])) throw Failure{RPD_E_INVALID, "alpha is NaN"};
  if (std::isnan(sigma)) throw Failure{RPD_E_INVALID, "sigma is NaN"};
  if ((ne && !keep_e) || (nf && !keep_f) || (nt && !keep_t)) throw Failure{RPD_E_INVALID, "null output mask"};

  // boundary incidences: the 4 triangles of each tet, the 3 edges of each triangle
  std::vector<std::pair<long long, long long>> tri_tet, edge_tri;
  std::vector<long long> tet_tri(4 * (size_t)nt), tri_edge(3 * (size_t)nf);
  for (long long t = 0; t < nt; ++t) {
    const int32_t* v = tets + 4 * t;
    for (int o = 0; o < 4; ++o) {  // the face opposite vertex o
      int32_t key[3];
      for (int c = 0, w = 0; c < 4; ++c)
        if (c != o) key[w++] = v[c];
      long long f = find_key<3>(tris, nf, key);
      if (f < 0) throw Failure{RPD_E_INVALID, "a face of a tet is not among the triangles"};
      tet_tri[4 * t + o] = f;
      tri_tet.push_back({f, t});
    }
  }
  for (long long f = 0; f < nf; ++f) {
    const int32_t* v = tris + 3 * f;
    for (int o = 0; o < 3; ++o) {
      int32_t key[2];
      for (int c = 0, w = 0; c < 3; ++c)
        if (c != o) key[w++] = v[c];
      long long e = find_key<2>(edges, ne, key);
      if (e < 0) throw Failure{RPD_E_INVALID, "an edge of a triangle is not among the edges"};
      tri_edge[3 * f + o] = e;
      edge_tri.push_back({e, f});
    }
  }
  Csr f_tets, e_tris;
  f_tets.build(nf, tri_tet);
  e_tris.build(ne, edge_tri);

  std::vector<uint8_t> live_t(nt, 1), live_f(nf, 1), live_e(ne, 1), orig(nf, 0);
  std::vector<int> tcount(nf, 0), fcount(ne, 0);
  for (long long f = 0; f < nf; ++f) {
    tcount[f] = (int)(f_tets.off[f + 1] - f_tets.off[f]);
    orig[f] = tcount[f] > 0;
  }
  for (long long e = 0; e < ne; ++e) fcount[e] = (int)(e_tris.off[e + 1] - e_tris.off[e]);

  // ---- tet-face pairs: (t, f) is simple when t is the only tet left on f; least alpha first (ties: lower f)
  typedef std::pair<double, long long> Item;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> q1;
  for (long long f = 0; f < nf; ++f)
    if (tcount[f] == 1) q1.push({alpha[f], f});
  while (!q1.empty()) {
    const long long f = q1.top().second;
    q1.pop();
    if (!live_f[f] || tcount[f] != 1) continue;
    long long t = -1;
    for (long long k = f_tets.off[f]; k < f_tets.off[f + 1]; ++k)
      if (live_t[f_tets.idx[k]]) t = f_tets.idx[k];
    live_t[t] = 0;
    live_f[f] = 0;
    for (int o = 0; o < 3; ++o) fcount[tri_edge[3 * f + o]]--;
    for (int o = 0; o < 4; ++o) {
      const long long g = tet_tri[4 * t + o];
      if (g == f) continue;
      if (--tcount[g] == 1) q1.push({alpha[g], g});
    }
  }

  // ---- face-edge pairs among the triangles of the original tets: (f, e) is simple when f is the only triangle
  //      left on e and no tet is left on f; least alpha first (ties: lower f, then lower e), while alpha < sigma
  typedef std::tuple<double, long long, long long> Item2;
  std::priority_queue<Item2, std::vector<Item2>, std::greater<Item2>> q2;
  auto offer = [&](long long e) {  // push the pair of e's only triangle, if it qualifies
    if (!live_e[e] || fcount[e] != 1) return;
    for (long long k = e_tris.off[e]; k < e_tris.off[e + 1]; ++k) {
      const long long g = e_tris.idx[k];
      if (live_f[g]) {
        if (orig[g] && tcount[g] == 0) q2.push({alpha[g], g, e});
        return;
      }
    }
  };
  for (long long e = 0; e < ne; ++e) offer(e);
  while (!q2.empty()) {
    const Item2 it = q2.top();
    q2.pop();
    const long long f = std::get<1>(it), e = std::get<2>(it);
    if (!live_f[f] || !live_e[e] || fcount[e] != 1 || tcount[f] != 0) continue;
    if (!(std::get<0>(it) < sigma)) break;
    live_f[f] = 0;
    live_e[e] = 0;
    for (int o = 0; o < 3; ++o) {
      const long long e2 = tri_edge[3 * f + o];
      if (e2 == e) continue;
      fcount[e2]--;
      offer(e2);
    }
  }
  std::memcpy(keep_e, live_e.data(), (size_t)ne);
  std::memcpy(keep_f, live_f.data(), (size_t)nf);
  std::memcpy(keep_t, live_t.data(), (size_t)nt);
}

}  // namespace rpd

extern "C" rpd_status rpd_thin(int32_t n_vertices, int64_t n_edges, const int32_t* edges, int64_t n_tris,
                               const int32_t* tris, const double* alpha, int64_t n_tets, const int32_t* tets,
                               double sigma, uint8_t* keep_edge, uint8_t* keep_tri, uint8_t* keep_tet) {
  try {
    rpd::thin(n_vertices, n_edges, edges, n_tris, tris, alpha, n_tets, tets, sigma, keep_edge, keep_tri, keep_tet);
    return RPD_OK;
  } catch (const rpd::Failure& f) {
    rpd::set_error(f.msg);
    return f.code;
  } catch (const std::bad_alloc&) {
    rpd::set_error("host allocation failed");
    return RPD_E_NOMEM;
  }
}
