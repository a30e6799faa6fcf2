// Tet-Cell clipping (paper Sec. 5.2) with on-the-fly fractional Euler characteristic (Sec. 4.1.2) and the gluing
// information for connected components (Sec. 4.1.1).
//
// Fast kernel: one workgroup owns TB spatially consecutive tets. It (1) selects the sites that can own any point of
// the group's bounding box, (2) selects per tet the candidate sites that can own a point of the tet, sorted by power
// distance at the tet centroid, (3) clips every (tet, candidate) piece by the bisectors of all other candidates, one
// thread per piece with the polytope in LDS, and (4) emits the piece's volume, moments, chi numerators and gluing
// bits. Pieces that do not fit (too many candidates or vertices) or whose predicates stay undecided in FP64 are
// deferred to the large-capacity kernel, which recomputes them with FP64 constructions and exact predicates.
#include <hip/hip_runtime.h>

#include <climits>

#include <algorithm>

#include "rpd_device.h"
#include "rpd_launch.h"

namespace rpd {

// ---------------------------------------------------------------------------------------------------------------
// emission of one nonempty piece
// ---------------------------------------------------------------------------------------------------------------
template <typename Topo>
__device__ inline int pos_of(typename Topo::W w, int p) {
  if (Topo::plane(w, 0) == p) return 0;
  if (Topo::plane(w, 1) == p) return 1;
  if (Topo::plane(w, 2) == p) return 2;
  return -1;
}

template <typename Topo>
__device__ inline long long wv_of(typename Topo::W w, const unsigned* nu, long long L) {
  return w_vertex(Topo::plane(w, 0), Topo::plane(w, 1), Topo::plane(w, 2), nu, L);
}

// One element piece (element, tet) is emitted exactly once per shape: adding sets its gluing bits and count,
// removing (the same piece recomputed from the state before an incremental update, sign -1) takes both back.
// The two happen in one launch, in either order. Each records the piece's gluing bits in its own half of the
// piece's tag pair; a scan after the launch flags the element for a new union-find only where the two differ (a
// piece put back with the same gluing bits leaves the element's forest as it was).
__device__ inline void node_emit(const ShapeArgs& a, int sign, unsigned long long key, int glue) {
  int ns = node_insert(a.N, key, a.status);
  if (ns < 0) return;
  atomicAdd(&a.N.rec[ns].st, sign * (NODE_UNIT + glue));  // removal re-emits the same bits, so this is exact
  if (a.touch_cell) a.removed[2 * (size_t)ns + (sign > 0)] = (unsigned short)(0x100 | glue);
}

// a per-piece element term for sampled comparisons (RPD_KEEP_PIECES only)
__device__ inline void keep_term(const ShapeArgs& a, int kind, int t, int i, int j, int k, int l, int glue,
                                 long long num) {
  if (!(a.flags & RPD_KEEP_PIECES)) return;
  const unsigned long long idx = atomicAdd(&a.counters[C_TERMS], 1ull);
  if (idx < (unsigned long long)a.term_cap) {
    TermRec r;
    r.kind = kind;
    r.t = t;
    r.i = i;
    r.j = j;
    r.k = k;
    r.l = l;
    r.glue = glue;
    r.pad = 0;
    r.num = num;
    a.terms[idx] = r;
  } else {
    atomicOr(a.status, ST_TABLE_FULL);
  }
}

// Hands a tet's sorted candidates (list positions into the workgroup's site list) to the large-capacity kernel;
// returns the item's list word (64 x list index + m), or 0 when the list buffer is full (the call is then redone
// with larger buffers, so no item is ever processed without its list).
__device__ inline int hand_over_list(const ShapeArgs& a, const unsigned char* cand, const int* sid, int m) {
  const unsigned long long idx = atomicAdd(&a.counters[C_LISTS], 1ull);
  if (idx >= (unsigned long long)a.list_cap) {
    atomicOr(a.status, ST_TABLE_FULL);
    return 0;
  }
  int* dst = a.deferred_list + idx * (size_t)KRAW;
  for (int c = 0; c < m; ++c) dst[c] = sid[cand[c]];
  return (int)(idx * 64) + m;
}

// The next chunk of a split item: the next tet while tets are taken one at a time (up to single_end), else the next
// SUB tets. False past the item's last tet.
__device__ inline bool next_chunk(int& sub, int& sub_n, int& single_end, int ntb_all) {
  if (single_end > sub + 1) {
    sub += 1;
    sub_n = 1;
    return true;
  }
  if (single_end > sub) {  // the last single tet of its chunk: on with the chunk after it
    sub = single_end;
    single_end = 0;
  } else {
    sub += SUB;
  }
  if (sub >= ntb_all) return false;
  sub_n = min(SUB, ntb_all - sub);
  return true;
}

// The environment of the fast kernel's piece (tet t, candidate ci of the tet's candidate bytes) in its shared lists.
__device__ inline void fast_env(TetEnv& env, const ShapeDesc& sd, int t, const float4* sites, const int* sid,
                                const unsigned char* cand, int ci) {
  env.tv = sd.tp + 4 * (size_t)t;
  env.o = env.tv[0];
  env.face64 = sd.tf + 4 * (size_t)t;
  env.sites = sites;
  env.sid = sid;
  env.cidx8 = cand;
  env.cidx32 = nullptr;
  env.csite = nullptr;
  env.ncs = 0;
  env.ci = ci;
  env.si = sites[cand[ci]];
  env.site_i = sid[cand[ci]];
}

// Hands a piece (tet t of the shape, site) with its tet's candidates to the large-capacity kernel.
__device__ inline void defer_piece(const ShapeArgs& a, int shape, int t, int site, const unsigned char* cand,
                                   const int* sid, int m) {
  stat_add(a, C_DEFER_CLIP, 1ull);
  const int list = hand_over_list(a, cand, sid, m);
  unsigned long long idx = atomicAdd(&a.counters[C_DEFER_ITEMS], 1ull);
  if (idx < (unsigned long long)a.deferred_cap) a.deferred[idx] = make_int4(shape, t, site, list);
  else atomicOr(a.status, ST_TABLE_FULL);
}

__device__ inline long long fixed56(double v) { return llrint(v * 72057594037927936.0); }  // 2^-56 units

// Cell volumes and first moments are exact sums of 128-bit integers in units of 2^-80 (resolution 8e-25, range
// 2^47), so that a nonempty piece far smaller than a grid cell still counts, every sum is independent of the order
// of the additions, and a removal pass takes its contributions back exactly. An accumulator is a (low, high) pair
// of 64-bit words; an addition adds the low word atomically and carries into the high word only when needed.
struct Fix128 {
  unsigned long long lo;
  long long hi;
};
__device__ inline Fix128 fixed80(double v) {
  const double D = rint(ldexp(v, 80));  // exact scaling, then the nearest integer
  const double h = floor(ldexp(D, -64));
  const double l = D - ldexp(h, 64);    // in [0, 2^64): the low bits of D, exact
  return Fix128{(unsigned long long)l, (long long)h};
}
__device__ inline Fix128 signed128(Fix128 x, int sign) {
  if (sign > 0) return x;
  return Fix128{0ull - x.lo, -x.hi - (x.lo != 0ull ? 1 : 0)};
}
__device__ inline void acc128(unsigned long long* p, Fix128 v) {
  const unsigned long long old = atomicAdd(p, v.lo);
  const long long h = v.hi + (old + v.lo < old ? 1 : 0);  // carry out of the low word
  if (h) atomicAdd(p + 1, (unsigned long long)h);
}

// Workgroup-local sums of the cell terms (chi numerator, piece count, fixed-point volume and moments) in n slots,
// each holding one site of the workgroup's list; a piece whose site has no slot adds to the global arrays directly.
struct CellSink {
  long long* chi;  // [n] (LDS)
  int* np;         // [n]
  unsigned long long* geo_lo;  // [4 n] low words of the workgroup's 128-bit sums
  int* geo_hi;                 // [4 n] their high words (a workgroup's sum stays below 2^84: 32 bits suffice)
  int n;
  int q;           // the slot of the piece's site, or -1 or >= n: none
};

template <typename T, typename Topo, typename Mask, int VCAP, bool EXACT, typename Tab>
__device__ __forceinline__ void emit_piece(Clipper<T, Topo, Mask, VCAP, EXACT, Tab>& c, const ShapeDesc& sd, int tl, const ShapeArgs& a,
                           const CellSink& sink) {
  typedef typename Topo::W W;
  const int i = c.env.site_i;  // batch-global site id
  const unsigned* nu = sd.nu + 14 * (size_t)tl;
  const long long L = sd.L;
  const int4 tn4 = reinterpret_cast<const int4*>(sd.tn)[tl];  // face neighbours (-1: boundary), one load
  const unsigned interior = (tn4.x >= 0 ? 1u : 0u) | (tn4.y >= 0 ? 2u : 0u) | (tn4.z >= 0 ? 4u : 0u) |
                            (tn4.w >= 0 ? 8u : 0u);  // bit f: face f is shared with another tet
  const int t = (int)(sd.tet_off + tl);  // batch-global tet id (node keys, piece records)
  const int sign = sd.sign;
  int* status = a.status;

  // ---- vertex pass: vertex and edge weights, face references, apex, RPVs
  long long sv = 0, se = 0;
  T gx = 0, gy = 0, gz = 0;
  int nv = 0;
  for (Mask m = c.live; m; m &= m - 1) {
    int k = ctz_mask(m);
    W w = c.st.topo(k);
    auto v = c.st.get(k);
    gx += v.x;
    gy += v.y;
    gz += v.z;
    ++nv;
    int p0 = Topo::plane(w, 0), p1 = Topo::plane(w, 1), p2 = Topo::plane(w, 2);
    sv += w_vertex(p0, p1, p2, nu, L);
    for (int e = 0; e < 3; ++e) {
      int nb = Topo::nb(w, e);
      if (k < nb) se += w_edge(Topo::plane(w, (e + 1) % 3), Topo::plane(w, (e + 2) % 3), nu, L);
      int p = Topo::plane(w, e);
      if (c.tab.get(p) == 0) c.tab.set(p, k + 1);
    }
    if (p0 >= 4 && p1 >= 4 && p2 >= 4) {
      int s0 = c.env.plane_site(p0), s1 = c.env.plane_site(p1), s2 = c.env.plane_site(p2);
      if (s0 > i && s1 > i && s2 > i) {  // the RPV is recorded once, from its smallest site
        int lo = min(s0, min(s1, s2)), hi = max(s0, max(s1, s2)), mid = s0 + s1 + s2 - lo - hi;
        unsigned long long ekey = ((unsigned long long)i << 42) | ((unsigned long long)lo << 21) | (unsigned)mid;
        int es = ht_insert(a.E, ekey, status);
        if (es >= 0) {
          int qs = ht_insert(a.Q, ((unsigned long long)es << 21) | (unsigned)hi, status);
          if (qs >= 0) atomicAdd(&a.rpv_cnt[qs], sign);
        }
        stat_add(a, C_RPV, 1ull);
        keep_term(a, 4, t, i, lo, mid, hi, 0, 1);
      }
    }
  }
  const T inv_nv = T(1) / T(nv);
  const T ax = gx * inv_nv, ay = gy * inv_nv, az = gz * inv_nv;

  // ---- face pass: face weights, cell gluing, face cycles (volume fans, RPF and RPE terms)
  long long sf = 0;
  int cell_glue = 0;
  T vol = 0, mx = 0, my = 0, mz = 0;
  for (int p = 0; p < c.np; ++p) {
    int r = c.tab.get(p);
    if (r == 0) continue;
    c.tab.set(p, 0);
    r -= 1;
    sf += (p < 4) ? (long long)nu[10 + p] : L;
    if (p < 4) cell_glue |= ((interior >> p) & 1u) ? 1 << p : 16 << p;  // glue across an interior face; boundary contact
    const int sp = c.env.plane_site(p);
    const bool felem = (p >= 4) && (sp > i);
    long long fv = 0, fe = 0;
    int fglue = 0;
    W wr = c.st.topo(r);
    auto R = c.st.get(r);
    int ep = pos_of<Topo>(wr, p);
    if (ep < 0) {
      atomicOr(status, ST_INTERNAL);
      continue;
    }
    int acur = Topo::plane(wr, (ep + 1) % 3);
    int nxt = Topo::nb(wr, (ep + 2) % 3);
    int cur = r;
    W wcur = wr;
    auto C = R;
    if (felem) fv += wv_of<Topo>(wr, nu, L);
    bool closed = false;
    for (int step = 0; step <= VCAP; ++step) {
      W wn = c.st.topo(nxt);
      auto N = c.st.get(nxt);
      int ea = pos_of<Topo>(wn, acur), epn = pos_of<Topo>(wn, p);
      if (ea < 0 || epn < 0) break;
      if (felem) {  // the edge cur -> nxt lies on planes {p, acur}
        fe += w_edge(p, acur, nu, L);
        if (acur < 4) {
          if ((interior >> acur) & 1u) fglue |= 1 << acur;
        } else if (acur > p) {
          int sa = c.env.plane_site(acur);
          if (sa > i) {  // RPE piece of {i, sp, sa}, counted from its smaller plane id
            int e1 = pos_of<Topo>(wcur, p), e2 = pos_of<Topo>(wcur, acur);
            int t1 = Topo::plane(wcur, 3 - e1 - e2);
            int t2 = Topo::plane(wn, 3 - ea - epn);
            long long ev = wv_of<Topo>(wcur, nu, L) + wv_of<Topo>(wn, nu, L) - L;
            int j = min(sp, sa), k = max(sp, sa);
            unsigned long long key = ((unsigned long long)i << 42) | ((unsigned long long)j << 21) | (unsigned)k;
            int es = ht_insert(a.E, key, status);
            if (es >= 0) {
              atomicAdd((unsigned long long*)&a.edge_chi[es], (unsigned long long)(sign * ev));
              atomicAdd(&a.edge_np[es], sign);
              const T lx = N.x - C.x, ly = N.y - C.y, lz = N.z - C.z;
              const double len = (double)sqrt(lx * lx + ly * ly + lz * lz);
              atomicAdd((unsigned long long*)&a.edge_len[es], (unsigned long long)(sign * fixed56(len)));
              int g = ((t1 < 4 && ((interior >> t1) & 1u)) ? (1 << t1) : 0) |
                      ((t2 < 4 && ((interior >> t2) & 1u)) ? (1 << t2) : 0);
              node_emit(a, sign, node_key(3, es, t), g);
              keep_term(a, 3, t, i, j, k, -1, g, ev);
            }
          }
        }
      }
      if (nxt == r) {
        closed = true;
        break;
      }
      if (felem) fv += wv_of<Topo>(wn, nu, L);
      if (cur != r) {  // fan triangle (R, C, N) with the apex: a tet of the piece
        T ux = C.x - R.x, uy = C.y - R.y, uz = C.z - R.z;
        T vx = N.x - R.x, vy = N.y - R.y, vz = N.z - R.z;
        T wx = ax - R.x, wy = ay - R.y, wz = az - R.z;
        T det = ux * (vy * wz - vz * wy) - uy * (vx * wz - vz * wx) + uz * (vx * wy - vy * wx);
        T tv = fabs(det) * T(1.0 / 6.0);
        vol += tv;
        mx += tv * (R.x + C.x + N.x + ax);
        my += tv * (R.y + C.y + N.y + ay);
        mz += tv * (R.z + C.z + N.z + az);
      }
      int ec = 3 - ea - epn;
      int c3 = Topo::plane(wn, ec);
      int nn = Topo::nb(wn, ea);  // leave nxt along {p, c3}: the neighbour opposite acur
      cur = nxt;
      wcur = wn;
      C = N;
      acur = c3;
      nxt = nn;
    }
    if (!closed) {
      atomicOr(status, ST_INTERNAL);
      continue;
    }
    if (felem) {
      long long fvl = fv - fe + L;
      unsigned long long key = ((unsigned long long)i << 32) | (unsigned)sp;
      int fs = ht_insert(a.F, key, status);
      if (fs >= 0) {
        atomicAdd((unsigned long long*)&a.face_chi[fs], (unsigned long long)(sign * fvl));
        atomicAdd(&a.face_np[fs], sign);
        node_emit(a, sign, node_key(2, fs, t), fglue);
      }
      keep_term(a, 2, t, i, sp, -1, -1, fglue, fvl);
    }
  }
  // ---- cell contributions
  long long chi = sv - se + sf - L;
  node_emit(a, sign, node_key(1, i, t), cell_glue);
  keep_term(a, 1, t, i, -1, -1, -1, cell_glue, chi);
  // moments were accumulated with 4x the centroid sum; shift to absolute coordinates
  const float4 o = c.env.o;
  double dvol = (double)vol;
  double dmx = (double)mx * 0.25 + dvol * o.x, dmy = (double)my * 0.25 + dvol * o.y,
         dmz = (double)mz * 0.25 + dvol * o.z;
  const Fix128 g[4] = {fixed80(dvol), fixed80(dmx), fixed80(dmy), fixed80(dmz)};
  if (sink.q >= 0 && sink.q < sink.n) {  // workgroup-local sums, flushed once per workgroup pass
    atomicAdd((unsigned long long*)&sink.chi[sink.q], (unsigned long long)chi);
    atomicAdd(&sink.np[sink.q], 1);
    for (int k = 0; k < 4; ++k) {
      const unsigned long long old = atomicAdd(&sink.geo_lo[4 * sink.q + k], g[k].lo);
      const long long h = g[k].hi + (old + g[k].lo < old ? 1 : 0);
      if (h) atomicAdd(&sink.geo_hi[4 * sink.q + k], (int)h);
    }
  } else {
    atomicAdd((unsigned long long*)&a.cell_chi[i], (unsigned long long)(sign * chi));
    atomicAdd(&a.cell_np[i], sign);
    for (int k = 0; k < 4; ++k)
      acc128((unsigned long long*)&a.cell_geo[2 * (4 * (size_t)i + k)], signed128(g[k], sign));
  }
  if (a.flags & RPD_KEEP_PIECES) {
    unsigned long long idx = atomicAdd(&a.counters[C_PIECES], 1ull);
    if (idx < (unsigned long long)a.piece_cap) {
      PieceRec pr;
      pr.t = t;
      pr.i = i;
      pr.vol = (float)dvol;
      pr.mx = (float)dmx;
      pr.my = (float)dmy;
      pr.mz = (float)dmz;
      pr.chi = chi;
      a.pieces[idx] = pr;
    } else {
      atomicOr(status, ST_TABLE_FULL);
    }
  }
}

// ---------------------------------------------------------------------------------------------------------------
// clipping of one (tet, candidate) piece against the other candidates in order; returns CLIP_* for the piece
// ---------------------------------------------------------------------------------------------------------------
template <typename T, typename Topo, typename Mask, int VCAP, bool EXACT, typename Tab>
__device__ __forceinline__ int clip_piece(Clipper<T, Topo, Mask, VCAP, EXACT, Tab>& cl, int m, int* status) {
  const TetEnv& env = cl.env;
  const float4 o = env.o;
  const double y1x = (double)env.tv[1].x - o.x, y1y = (double)env.tv[1].y - o.y, y1z = (double)env.tv[1].z - o.z;
  const double y2x = (double)env.tv[2].x - o.x, y2y = (double)env.tv[2].y - o.y, y2z = (double)env.tv[2].z - o.z;
  const double y3x = (double)env.tv[3].x - o.x, y3y = (double)env.tv[3].y - o.y, y3z = (double)env.tv[3].z - o.z;
  cl.init_tet();
  for (int c = 0; c < m; ++c) {
    if (c == env.ci) continue;
    float4 sj = env.cand_site(c);
    Plane<double> P = bisector64(env.si, sj, o);
    if (P.nx == 0.0 && P.ny == 0.0 && P.nz == 0.0) {  // concentric spheres: the larger one owns everything
      if (P.d > 0) continue;
      // equal spheres: under the weight perturbation eps_i - eps_j the lower site id owns everything
      if (P.d == 0 && env.site_i < env.cand_id(c)) continue;
      return CLIP_EMPTY;
    }
    // the bisector's values at the tet vertices are exact in FP64
    double h0 = P.d;
    double h1 = fma(P.nx, y1x, fma(P.ny, y1y, fma(P.nz, y1z, P.d)));
    double h2 = fma(P.nx, y2x, fma(P.ny, y2y, fma(P.nz, y2z, P.d)));
    double h3 = fma(P.nx, y3x, fma(P.ny, y3y, fma(P.nz, y3z, P.d)));
    if (h0 > 0 && h1 > 0 && h2 > 0 && h3 > 0) continue;  // the tet lies in H_ij: no cut
    if (h0 < 0 && h1 < 0 && h2 < 0 && h3 < 0) return CLIP_EMPTY;
    int r = cl.clip(4 + c, round_plane<T>(P));
    if (r != CLIP_OK) return r;
  }
  return CLIP_OK;
}

// ---------------------------------------------------------------------------------------------------------------
// fast kernel
// ---------------------------------------------------------------------------------------------------------------
__device__ inline double wave_min(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}
__device__ inline float wave_minf(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
  return v;
}
__device__ inline float wave_maxf(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

// g_j at the four tet vertices (tet-local frame, exact in FP64)
__device__ __forceinline__ void g4(const float4* tv, const float4& s, double* g) {
  const float4 o = tv[0];
  double ax = (double)s.x - o.x, ay = (double)s.y - o.y, az = (double)s.z - o.z;
  double D = ax * ax + ay * ay + az * az - (double)s.w * s.w;
  g[0] = D;
  for (int v = 1; v < 4; ++v)
    g[v] = D - 2.0 * (((double)tv[v].x - o.x) * ax + ((double)tv[v].y - o.y) * ay + ((double)tv[v].z - o.z) * az);
}

// Remove candidates dominated on the whole tet by one of the first three candidates (exact test: g_j - g_i is
// affine, so being larger at the four vertices means larger everywhere on the tet and j owns no point of it).
// The list must be sorted (only_count: the list is unsorted and over budget; it is filtered but stays unsorted).
// Drops the candidates that another candidate beats at all four tet vertices (g is affine, so then everywhere on the
// tet: the site owns nothing there and its bisector constrains no piece; the values are exact in FP64). The list is
// sorted by the power distance at the centroid, and a dominator has the smaller one, so rounds of three dominators
// taken in list order (each tested against the candidates after them) find the dominated candidates the three-at-a-time
// way; the rounds run while candidates remain past the dominators. Returns the new count; order is kept.
__device__ __forceinline__ int refine_candidates(const float4* tv, const float4* sites, unsigned char* cand, float* key,
                                                 int m) {
  for (int d = 0; d + 3 < m; d += 3) {
    double g0[4], g1[4], g2[4];
    g4(tv, sites[cand[d]], g0);
    g4(tv, sites[cand[d + 1]], g1);
    g4(tv, sites[cand[d + 2]], g2);
    int w = d + 3;
    for (int c = d + 3; c < m; ++c) {
      double g[4];
      g4(tv, sites[cand[c]], g);
      const bool dom = (g[0] > g0[0] && g[1] > g0[1] && g[2] > g0[2] && g[3] > g0[3]) ||
                       (g[0] > g1[0] && g[1] > g1[1] && g[2] > g1[2] && g[3] > g1[3]) ||
                       (g[0] > g2[0] && g[1] > g2[1] && g[2] > g2[2] && g[3] > g2[3]);
      if (!dom) {
        cand[w] = cand[c];
        key[w] = key[c];
        ++w;
      }
    }
    m = w;
  }
  return m;
}

// Two LDS layouts of the fast kernel (64 threads). With 16 vertex slots per piece, 256 sites in the shared list, 40
// raw candidates per tet and the cell sums of 32 sites, a workgroup takes about 27 KB and six fit a compute unit; with
// 12 slots, 192 sites, 36 raw candidates and the sums of 16 sites it takes under 20 KB and eight fit (two waves per
// SIMD). Pieces that outgrow their slots are redone inside the kernel with the 64-slot polytope, and a tet's path to
// the large-capacity kernel depends on its own candidates only, so both layouts give the same elements; the 12-slot
// one redoes more pieces and splits more blocks, and wins where occupancy, not the longest items, bounds the kernel.
template <int SLOTS>
struct FastCfg;
template <>
struct FastCfg<16> {
  static constexpr int VCAP = 16, SL = 256, KR = 40, AGG64 = 32;
  static constexpr bool USED_FIRST = false;
};
template <>
struct FastCfg<12> {
  static constexpr int VCAP = 12, SL = 192, KR = 36, AGG64 = 16;
  static constexpr bool USED_FIRST = true;
};

template <typename T, int NT, int SLOTS>
__global__ __launch_bounds__(NT) void k_clip_fast(ShapeArgs a) {
  typedef FastCfg<SLOTS> FC;
  constexpr int SLMAX = FC::SL, KRAW = FC::KR, VMAX = FC::VCAP;
  static_assert(KRAW <= rpd::KRAW && SLMAX <= 256, "candidate bytes index the site list; hand-over lists hold rpd::KRAW");
  static_assert(NT % TB == 0 && NT >= TB, "threads per block must be a multiple of the tets per block");
  constexpr int TPT = NT / TB;  // threads per tet in the candidate phase
  __shared__ float4 s_site[SLMAX];
  __shared__ int s_sid[SLMAX];
  __shared__ unsigned char s_cand[TB][KRAW];
  // the candidates' sort keys are dead before the clipping phase starts: they share storage with the polytopes
  typedef typename StoreOf<T, Topo32, VMAX>::type PolyStore;
  constexpr size_t XYZ_BYTES = PolyStore::coord_bytes(NT);
  constexpr size_t KEY_BYTES = sizeof(float) * TB * KRAW;
  __shared__ __attribute__((aligned(16))) unsigned char s_share[XYZ_BYTES > KEY_BYTES ? XYZ_BYTES : KEY_BYTES];
  float(*s_key)[KRAW] = reinterpret_cast<float(*)[KRAW]>(s_share);
  __shared__ int s_m[TB];
  static_assert(TB * KMAX < 32768, "piece offsets are 16-bit");
  __shared__ short s_off[TB + 1];
  __shared__ short s_order[TB];
  __shared__ float s_box[6];
  __shared__ double s_red[NT / 64];
  __shared__ int s_nsl;
  __shared__ unsigned long long s_cnt[4];
  __shared__ unsigned s_topo[VMAX * NT];
  __shared__ int s_over[NT];  // this round's pieces that ran out of vertex slots: tet << 16 | candidate
  __shared__ int s_nover;
  // per-site sums of the workgroup's cell terms (the first 128 sites of the list, or the first 32 with 64 threads,
  // where the LDS budget for four workgroups per compute unit is tight); pieces of later sites add to the global
  // accumulators directly
  constexpr int AGG = NT == 64 ? FC::AGG64 : 128;
  __shared__ long long s_acc_chi[AGG];
  __shared__ int s_acc_np[AGG];
  __shared__ unsigned long long s_acc_lo[4 * AGG];
  __shared__ int s_acc_hi[4 * AGG];
  // the sums' slot of each site of the list (255: none): with USED_FIRST, the sites that are candidates of a tet
  // clipped here take the first AGG slots in list order, so that the few sums cover the sites that own the pieces;
  // else slot q holds list position q (no map: its bytes would cost the 16-slot layout its sixth workgroup)
  constexpr bool UF = FC::USED_FIRST;
  __shared__ unsigned char s_agg[UF ? SLMAX : 1];
  __shared__ unsigned char s_aggq[UF ? AGG : 1];  // the list position of each slot's site
  __shared__ int s_nagg;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  if (tid == 0) s_nover = 0;
  for (int k = tid; k < AGG; k += NT) {
    s_acc_chi[k] = 0;
    s_acc_np[k] = 0;
    for (int d = 0; d < 4; ++d) {
      s_acc_lo[4 * k + d] = 0;
      s_acc_hi[4 * k + d] = 0;
    }
  }
  unsigned long long n_pairs = 0, n64 = 0, n_cand = 0;
  const int nitems = a.nitems_dev ? *a.nitems_dev : a.nitems;
  // Work items are (shape, block or part of a block), ordered heaviest first. In a build the grid covers them, one
  // item per workgroup, and the hardware dispatcher hands them to compute units in that order as they free up,
  // which is the work queue. The passes of an incremental round read the item count on the device and launch a
  // grid sized to the resident workgroups, each taking items in grid-stride order.
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
  const unsigned long long clock0 = wall_clock64();
  const int2 wi = a.items[item];
  const int shape = __builtin_amdgcn_readfirstlane(wi.x & 0xffff);
  const ShapeDesc sd = a.shapes[shape];
  const int blk = wi.y & ((1 << ITEM_PART_SHIFT) - 1), part = wi.y >> ITEM_PART_SHIFT;
  // the tets of the item to clip, relative to its first tet (an incremental update names the tets a new sphere can
  // reach; every other item takes all)
  const unsigned tet_mask16 = (unsigned)wi.x >> 16;
  const unsigned long long item_mask = tet_mask16 ? (unsigned long long)tet_mask16 : ~0ull;
  int tb0 = sd.blk[blk];
  int ntb_all = sd.blk[blk + 1] - tb0;
  if (part > 0) {  // one part of a heavy block (the host only makes parts that exist)
    tb0 += (part - 1) * SPLIT_TETS;
    ntb_all = min(SPLIT_TETS, ntb_all - (part - 1) * SPLIT_TETS);
  }
  // A block whose shared site list overflows is redone in chunks of SUB tets (smaller boxes, shorter lists), and a
  // chunk that still overflows one tet at a time, each with its own candidates found among all of the shape's
  // sites. A tet then goes to the large-capacity kernel only for reasons that depend on its own candidates (more
  // than fit the list, or the clip budget), never on its neighbours' or on sites that own nothing in it: an
  // incremental update, which recomputes a tet's pieces to take them back, must take the path that added them.
  int sub = 0, sub_n = ntb_all, single_end = 0;  // tets [sub, single_end): one at a time
  bool split = false;
  while (true) {
  const int t0 = tb0 + sub;
  const int ntb = sub_n;
  const bool single = single_end > sub;
  const unsigned long long cmask = item_mask >> sub;  // bit lt: tet t0 + lt is clipped
  if (split && !(cmask & (ntb >= 64 ? ~0ull : (1ull << ntb) - 1ull))) {  // a chunk without such tets
    if (!next_chunk(sub, sub_n, single_end, ntb_all)) break;
    continue;
  }
  int tpt = TPT;  // threads per tet in the candidate phase
  while (tpt < 64 && 2 * tpt * ntb <= NT) tpt *= 2;

  // ---- 1. the tets' bounding box (tet vertices and face planes are read from HBM where they are needed, through
  //        the caches: on chip, the LDS budget goes to the polytopes, so that more workgroups fit a compute unit)
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (tid < TB) {
    if (!single && tid < ntb && ((cmask >> tid) & 1ull)) {
      const float4* tp = sd.tp + 4 * (size_t)(t0 + tid);
      for (int v = 0; v < 4; ++v) {
        float4 p = tp[v];
        lo[0] = fminf(lo[0], p.x);
        lo[1] = fminf(lo[1], p.y);
        lo[2] = fminf(lo[2], p.z);
        hi[0] = fmaxf(hi[0], p.x);
        hi[1] = fmaxf(hi[1], p.y);
        hi[2] = fmaxf(hi[2], p.z);
      }
    }
    s_m[tid] = 0;
    for (int k = 0; k < 3; ++k) {
      float l = wave_minf(lo[k]), h = wave_maxf(hi[k]);
      if (tid == 0) {
        s_box[k] = l;
        s_box[3 + k] = h;
      }
    }
  }
  if (tid == 0) s_nsl = 0;
  __syncthreads();

  // ---- 2. sites that can own a point of the box: min over the box of g_j <= min over j of max over the box
  //        (g_j(x) = d_j(x) - |x - o|^2 is affine; values exact in FP64); for a single tet, the same test on the
  //        tet itself (its exact candidates)
  const float4* ssite = a.site + sd.site_off;
  if (single) {
    const float4* tv = sd.tp + 4 * (size_t)t0;
    const float4 o = tv[0];
    double y[3][3];
    for (int v = 1; v < 4; ++v) {
      y[v - 1][0] = (double)tv[v].x - o.x;
      y[v - 1][1] = (double)tv[v].y - o.y;
      y[v - 1][2] = (double)tv[v].z - o.z;
    }
    // the five dominators of the candidate phase among all of the shape's sites (lowest index on ties): the site
    // attaining U and the owner of each vertex; a site one of them beats at all four vertices is not collected, so
    // that the list holds the tet's exact candidates less those (which the candidate phase drops anyway)
    double dv[5];
    int dj[5];
    for (int k = 0; k < 5; ++k) {
      dv[k] = INFINITY;
      dj[k] = 0x7fffffff;
    }
    for (int j = tid; j < sd.ns; j += NT) {
      const float4 s = ssite[j];
      const double ax_ = (double)s.x - o.x, ay_ = (double)s.y - o.y, az_ = (double)s.z - o.z;
      double gq[4];
      gq[0] = ax_ * ax_ + ay_ * ay_ + az_ * az_ - (double)s.w * s.w;
      for (int v = 0; v < 3; ++v) gq[v + 1] = gq[0] - 2.0 * (y[v][0] * ax_ + y[v][1] * ay_ + y[v][2] * az_);
      const double gmx = fmax(fmax(gq[0], gq[1]), fmax(gq[2], gq[3]));
      for (int k = 0; k < 5; ++k) {
        const double x = k == 0 ? gmx : gq[k - 1];
        if (x < dv[k] || (x == dv[k] && j < dj[k])) {
          dv[k] = x;
          dj[k] = j;
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1)
      for (int k = 0; k < 5; ++k) {
        const double x2 = __shfl_xor(dv[k], off);
        const int j2 = __shfl_xor(dj[k], off);
        if (x2 < dv[k] || (x2 == dv[k] && j2 < dj[k])) {
          dv[k] = x2;
          dj[k] = j2;
        }
      }
    if constexpr (NT > 64) {  // across the waves, through the polytope area (unused until the pieces)
      double* xv = reinterpret_cast<double*>(s_share);
      int* xj = reinterpret_cast<int*>(s_share + sizeof(double) * 5 * (NT / 64));
      if (lane == 0)
        for (int k = 0; k < 5; ++k) {
          xv[5 * wid + k] = dv[k];
          xj[5 * wid + k] = dj[k];
        }
      __syncthreads();
      for (int w = 0; w < NT / 64; ++w)
        for (int k = 0; k < 5; ++k) {
          const double x2 = xv[5 * w + k];
          const int j2 = xj[5 * w + k];
          if (x2 < dv[k] || (x2 == dv[k] && j2 < dj[k])) {
            dv[k] = x2;
            dj[k] = j2;
          }
        }
    }
    const double U = dv[0];
    double gb[5][4];
    for (int k = 0; k < 5; ++k) {
      const float4 s = ssite[dj[k]];
      const double ax_ = (double)s.x - o.x, ay_ = (double)s.y - o.y, az_ = (double)s.z - o.z;
      gb[k][0] = ax_ * ax_ + ay_ * ay_ + az_ * az_ - (double)s.w * s.w;
      for (int v = 0; v < 3; ++v) gb[k][v + 1] = gb[k][0] - 2.0 * (y[v][0] * ax_ + y[v][1] * ay_ + y[v][2] * az_);
    }
    for (int j = tid; j < sd.ns; j += NT) {
      const float4 s = ssite[j];
      const double ax_ = (double)s.x - o.x, ay_ = (double)s.y - o.y, az_ = (double)s.z - o.z;
      double g[4];
      g[0] = ax_ * ax_ + ay_ * ay_ + az_ * az_ - (double)s.w * s.w;
      for (int v = 0; v < 3; ++v) g[v + 1] = g[0] - 2.0 * (y[v][0] * ax_ + y[v][1] * ay_ + y[v][2] * az_);
      const double gmn = fmin(fmin(g[0], g[1]), fmin(g[2], g[3]));
      bool dom = false;
      for (int k = 0; k < 5; ++k)
        dom = dom || (g[0] > gb[k][0] && g[1] > gb[k][1] && g[2] > gb[k][2] && g[3] > gb[k][3]);
      if (gmn <= U && !dom) {
        const int q = atomicAdd(&s_nsl, 1);
        if (q < SLMAX) {
          s_site[q] = s;
          s_sid[q] = sd.site_off + j;
        }
      }
    }
  } else {
  const double bx = s_box[0], by = s_box[1], bz = s_box[2];
  const double ex = (double)s_box[3] - bx, ey = (double)s_box[4] - by, ez = (double)s_box[5] - bz;
  double umin = INFINITY;
  for (int j = tid; j < sd.ns; j += NT) {
    float4 s = ssite[j];
    double ax_ = (double)s.x - bx, ay_ = (double)s.y - by, az_ = (double)s.z - bz;
    double D = ax_ * ax_ + ay_ * ay_ + az_ * az_ - (double)s.w * s.w;
    double gmax = D + fmax(0.0, -2.0 * ex * ax_) + fmax(0.0, -2.0 * ey * ay_) + fmax(0.0, -2.0 * ez * az_);
    umin = fmin(umin, gmax);
  }
  umin = wave_min(umin);
  if (lane == 0) s_red[wid] = umin;
  __syncthreads();
  double UB = s_red[0];
  for (int w = 1; w < NT / 64; ++w) UB = fmin(UB, s_red[w]);
  for (int j = tid; j < sd.ns; j += NT) {
    float4 s = ssite[j];
    double ax_ = (double)s.x - bx, ay_ = (double)s.y - by, az_ = (double)s.z - bz;
    double D = ax_ * ax_ + ay_ * ay_ + az_ * az_ - (double)s.w * s.w;
    double gmin = D + fmin(0.0, -2.0 * ex * ax_) + fmin(0.0, -2.0 * ey * ay_) + fmin(0.0, -2.0 * ez * az_);
    if (gmin <= UB) {
      int q = atomicAdd(&s_nsl, 1);
      if (q < SLMAX) {
        s_site[q] = s;
        s_sid[q] = sd.site_off + j;
      }
    }
  }
  }
  __syncthreads();
  const int nsl = s_nsl;
  if (nsl > SLMAX && !(a.flags & RPD_FORCE_SLOW_PATH)) {
    if (!split && ntb > SUB) {  // chunks of SUB tets
      split = true;
      sub_n = SUB;
      if (tid == 0) stat_add(a, C_SPLIT, 1ull);
      __syncthreads();
      continue;
    }
    if (!single) {  // one tet at a time, each with its exact candidates
      split = true;
      single_end = sub + ntb;
      sub_n = 1;
      __syncthreads();
      continue;
    }
  }
  const bool block_overflow = nsl > SLMAX || (a.flags & RPD_FORCE_SLOW_PATH);
  if constexpr (UF)
    for (int q = tid; q < min(nsl, SLMAX); q += NT) s_agg[q] = 0;

  // ---- 3. candidates of every tet: sites whose minimum over the tet is <= min_j max over the tet
  if (!block_overflow) {
    const int lt = tid / tpt, h = tid % tpt;
    if (lt < ntb && ((cmask >> lt) & 1ull)) {
      const float4* tv = sd.tp + 4 * (size_t)(t0 + lt);
      const float4 o = tv[0];
      double y[3][3];
      for (int v = 1; v < 4; ++v) {
        y[v - 1][0] = (double)tv[v].x - o.x;
        y[v - 1][1] = (double)tv[v].y - o.y;
        y[v - 1][2] = (double)tv[v].z - o.z;
      }
      const double ycx = (y[0][0] + y[1][0] + y[2][0]) * 0.25, ycy = (y[0][1] + y[1][1] + y[2][1]) * 0.25,
                   ycz = (y[0][2] + y[1][2] + y[2][2]) * 0.25;
      // five dominators, each a site with its list position and id (the lowest id on ties, so that the choice does
      // not depend on the list's order): [0] attains U = min over sites of the maximum of g over the tet, [1 + v]
      // the minimum of g at vertex v (that vertex's owner)
      double dv[5];
      int dq[5], did[5];
      for (int k = 0; k < 5; ++k) {
        dv[k] = INFINITY;
        dq[k] = 0;
        did[k] = 0x7fffffff;
      }
      for (int q = h; q < nsl; q += tpt) {
        float4 s = s_site[q];
        double ax_ = (double)s.x - o.x, ay_ = (double)s.y - o.y, az_ = (double)s.z - o.z;
        double gq[4];
        gq[0] = ax_ * ax_ + ay_ * ay_ + az_ * az_ - (double)s.w * s.w;
        for (int v = 0; v < 3; ++v) gq[v + 1] = gq[0] - 2.0 * (y[v][0] * ax_ + y[v][1] * ay_ + y[v][2] * az_);
        const double gmx = fmax(fmax(gq[0], gq[1]), fmax(gq[2], gq[3]));
        const int id = s_sid[q];
        for (int k = 0; k < 5; ++k) {
          const double x = k == 0 ? gmx : gq[k - 1];
          if (x < dv[k] || (x == dv[k] && id < did[k])) {
            dv[k] = x;
            dq[k] = q;
            did[k] = id;
          }
        }
      }
      for (int off = 1; off < tpt; off <<= 1)
        for (int k = 0; k < 5; ++k) {
          const double x2 = __shfl_xor(dv[k], off);
          const int q2 = __shfl_xor(dq[k], off), id2 = __shfl_xor(did[k], off);
          if (x2 < dv[k] || (x2 == dv[k] && id2 < did[k])) {
            dv[k] = x2;
            dq[k] = q2;
            did[k] = id2;
          }
        }
      const double U = dv[0];
      if (a.tet_U && sd.sign > 0 && h == 0) a.tet_U[sd.tet_off + t0 + lt] = U;
      // the dominators' g at the four vertices: a site that one of them beats at all four owns no point of the tet
      // and its bisector constrains no piece (the dominator is a candidate, and its own bisector already does), so
      // it is not a candidate; the same test among all candidates follows once they are sorted
      double gb[5][4];
      for (int k = 0; k < 5; ++k) {
        const float4 s = s_site[dq[k]];
        const double ax_ = (double)s.x - o.x, ay_ = (double)s.y - o.y, az_ = (double)s.z - o.z;
        gb[k][0] = ax_ * ax_ + ay_ * ay_ + az_ * az_ - (double)s.w * s.w;
        for (int v = 0; v < 3; ++v) gb[k][v + 1] = gb[k][0] - 2.0 * (y[v][0] * ax_ + y[v][1] * ay_ + y[v][2] * az_);
      }
      for (int q = h; q < nsl; q += tpt) {
        float4 s = s_site[q];
        double ax_ = (double)s.x - o.x, ay_ = (double)s.y - o.y, az_ = (double)s.z - o.z;
        double g[4];
        g[0] = ax_ * ax_ + ay_ * ay_ + az_ * az_ - (double)s.w * s.w;
        for (int v = 0; v < 3; ++v) g[v + 1] = g[0] - 2.0 * (y[v][0] * ax_ + y[v][1] * ay_ + y[v][2] * az_);
        const double gmn = fmin(fmin(g[0], g[1]), fmin(g[2], g[3]));
        bool dom = false;
        for (int k = 0; k < 5; ++k)
          dom = dom || (g[0] > gb[k][0] && g[1] > gb[k][1] && g[2] > gb[k][2] && g[3] > gb[k][3]);
        const double D = g[0];
        if (gmn <= U && !dom) {
          int pos = atomicAdd(&s_m[lt], 1);
          if (pos < KRAW) {
            s_cand[lt][pos] = (unsigned char)q;
            s_key[lt][pos] = (float)(D - 2.0 * (ycx * ax_ + ycy * ay_ + ycz * az_));
          }
        }
      }
    }
  }
  __syncthreads();
  // sort each tet's candidates by (power distance at the centroid, site id), drop the dominated ones, and mark the
  // tets that keep more than the budget
  if (tid < ntb && ((cmask >> tid) & 1ull)) {
    int m = s_m[tid];
    if (!block_overflow && m <= KRAW) {
      for (int x = 1; x < m; ++x) {
        const float kx = s_key[tid][x];
        const unsigned char cx = s_cand[tid][x];
        const int ix = s_sid[cx];
        int y = x - 1;
        while (y >= 0 && (s_key[tid][y] > kx || (s_key[tid][y] == kx && s_sid[s_cand[tid][y]] > ix))) {
          s_key[tid][y + 1] = s_key[tid][y];
          s_cand[tid][y + 1] = s_cand[tid][y];
          --y;
        }
        s_key[tid][y + 1] = kx;
        s_cand[tid][y + 1] = cx;
      }
      m = refine_candidates(sd.tp + 4 * (size_t)(t0 + tid), s_site, s_cand[tid], s_key[tid], m);
    }
    if (block_overflow || m > a.kmax) {
      s_m[tid] = -1;
      stat_add(a, block_overflow ? C_DEFER_BLOCK : C_DEFER_KMAX, 1ull);
      // the sorted, refined candidates go with the tet when they fit the list (else the large-capacity kernel finds
      // them among all sites); either way the choice depends on the tet's candidates only
      const int list = (!block_overflow && m <= KRAW) ? hand_over_list(a, s_cand[tid], s_sid, m) : 0;
      unsigned long long idx = atomicAdd(&a.counters[C_DEFER_ITEMS], 1ull);
      if (idx < (unsigned long long)a.deferred_cap) a.deferred[idx] = make_int4(shape, t0 + tid, -1, list);
      else atomicOr(a.status, ST_TABLE_FULL);
    } else {
      s_m[tid] = m;
      if constexpr (UF)
        for (int x = 0; x < m; ++x) s_agg[s_cand[tid][x]] = 1;
    }
  }
  __syncthreads();
  // pieces are laid out tet by tet with the tets ordered by candidate count, largest first: every piece of a tet
  // loops over the same planes, so a wavefront's lanes then have similar trip counts
  if (tid < TB) {
    const int mt = tid < ntb ? max(s_m[tid], 0) : 0;
    int rank = 0;
    for (int u = 0; u < TB; ++u) {
      const int mu = u < ntb ? max(s_m[u], 0) : 0;
      rank += (mu > mt || (mu == mt && u < tid)) ? 1 : 0;
    }
    s_order[rank] = tid;
  }
  __syncthreads();
  if (wid == 0) {
    const int nl = min(nsl, SLMAX);
    int nagg = nl;
    if constexpr (UF) {
      nagg = 0;
      for (int c = 0; c < nl; c += 64) {
        const int q = c + lane;
        const bool used = q < nl && s_agg[q] != 0;
        const unsigned long long mk = __ballot(used);
        const int r = nagg + __popcll(mk & ((1ull << lane) - 1ull));
        if (q < nl) s_agg[q] = (used && r < AGG) ? (unsigned char)r : (unsigned char)255;
        if (used && r < AGG) s_aggq[r] = (unsigned char)q;
        nagg += __popcll(mk);
      }
    }
    if (lane == 0) s_nagg = min(nagg, AGG);
  }
  if (tid == 0) {
    int acc = 0;
    for (int j = 0; j < TB; ++j) {
      s_off[j] = acc;
      const int lt = s_order[j];
      if (lt < ntb && s_m[lt] > 0) acc += s_m[lt];
    }
    s_off[TB] = acc;
  }
  __syncthreads();

  // ---- 4. one thread per (tet, candidate) piece
  const int npairs = s_off[TB];
  n_cand += npairs;
  for (int base = 0; base < npairs; base += NT) {  // rounds of NT pieces (the same count for every thread)
    const int p = base + tid;
    if (p < npairs) {
      int lo_ = 0, hi_ = TB - 1;  // last position j with s_off[j] <= p
      while (lo_ < hi_) {
        int mid = (lo_ + hi_ + 1) >> 1;
        if (s_off[mid] <= p) lo_ = mid;
        else hi_ = mid - 1;
      }
      const int lt = s_order[lo_];
      const int ci = p - s_off[lo_];
      const int m = s_m[lt];
      Clipper<T, Topo32, unsigned, VMAX, false, RegTab> cl;
      cl.st.bind(s_share, s_topo, tid, NT);
      cl.tab.clear(0);
      cl.a = nullptr;  // only the exact predicates use it (not compiled into this kernel)
      cl.flags = a.flags;
      cl.np = 4 + m;
      cl.n64 = 0;
      cl.nex = 0;
      fast_env(cl.env, sd, t0 + lt, s_site, s_sid, s_cand[lt], ci);
      const int r = clip_piece(cl, m, a.status);
      n64 += cl.n64;
      if (r == CLIP_OK) {
        n_pairs += (unsigned long long)(long long)sd.sign;  // live pieces, in two's complement
        const int slot = UF ? (int)s_agg[s_cand[lt][ci]] : (int)s_cand[lt][ci];
        emit_piece(cl, sd, t0 + lt, a, CellSink{s_acc_chi, s_acc_np, s_acc_lo, s_acc_hi, AGG, slot});
      } else if (r == CLIP_DEFER) {
        defer_piece(a, shape, t0 + lt, cl.env.site_i, s_cand[lt], s_sid, m);
      } else if (r == CLIP_FULL) {  // out of vertex slots: redone below, after this round
        s_over[atomicAdd(&s_nover, 1)] = (lt << 16) | ci;
      }
    }
    // Pieces that ran out of vertex slots are redone here, one per thread, with a BIG_VCAP-slot polytope (they
    // would otherwise wait for the deferred kernel, after this one). The round's small polytopes are dead by now,
    // so the first records live in their LDS; more go to a global-memory pool (same arithmetic, same bits). Which
    // path computes a piece must depend on the piece alone (an incremental update must take back exactly the bits
    // it added), so a full pool is a table overflow (the call is redone with larger buffers), never a deferral.
    __syncthreads();
    const int nover = s_nover;
    if (nover) {
      if (tid < nover) {
        const int lt = s_over[tid] >> 16, ci = s_over[tid] & 0xffff, m = s_m[lt];
        constexpr size_t CB = sizeof(typename Coord4<T>::type) * BIG_VCAP;
        constexpr size_t REC = (CB + 8 * BIG_VCAP + 64 + 15) / 16 * 16;
        constexpr int NLDS = (int)(sizeof(s_share) / REC);
        static_assert(CB + 8 * BIG_VCAP + 32 <= BIG_BYTES, "large-capacity polytope record");
        const unsigned long long slot = atomicAdd(&a.counters[C_BIG], 1ull);
        if (tid >= NLDS && slot >= (unsigned long long)a.big_cap) {
          atomicOr(a.status, ST_TABLE_FULL);
        } else {
          unsigned char* b = tid < NLDS ? s_share + (size_t)tid * REC : a.big + slot * BIG_BYTES;
          Clipper<T, Topo64, unsigned long long, BIG_VCAP, false, MemTab> cb;
          cb.st.c = reinterpret_cast<typename Coord4<T>::type*>(b);
          cb.st.w = reinterpret_cast<unsigned long long*>(b + CB);
          cb.st.stride = 1;
          cb.tab.base = b + CB + 8 * BIG_VCAP;
          cb.tab.stride = 1;
          cb.tab.clear(4 + m);
          cb.a = nullptr;
          cb.flags = a.flags;
          cb.np = 4 + m;
          cb.n64 = 0;
          cb.nex = 0;
          fast_env(cb.env, sd, t0 + lt, s_site, s_sid, s_cand[lt], ci);
          const int r = clip_piece(cb, m, a.status);
          n64 += cb.n64;
          if (r == CLIP_OK) {
            n_pairs += (unsigned long long)(long long)sd.sign;
            const int slot = UF ? (int)s_agg[s_cand[lt][ci]] : (int)s_cand[lt][ci];
            emit_piece(cb, sd, t0 + lt, a, CellSink{s_acc_chi, s_acc_np, s_acc_lo, s_acc_hi, AGG, slot});
          } else if (r != CLIP_EMPTY) {  // a predicate undecided in FP64, or over BIG_VCAP vertices
            defer_piece(a, shape, t0 + lt, cb.env.site_i, s_cand[lt], s_sid, m);
          }
        }
      }
      __syncthreads();
      if (tid == 0) s_nover = 0;
      __syncthreads();
    }
  }
  // flush the workgroup's cell sums of this pass (the site list changes with the next chunk)
  __syncthreads();
  for (int q = tid; q < s_nagg; q += NT) {  // q: the slot
    const int np_q = s_acc_np[q];
    if (np_q == 0) continue;
    const int i = s_sid[UF ? (int)s_aggq[q] : q];
    atomicAdd((unsigned long long*)&a.cell_chi[i], (unsigned long long)(sd.sign * s_acc_chi[q]));
    atomicAdd(&a.cell_np[i], sd.sign * np_q);
    for (int d = 0; d < 4; ++d) {
      const Fix128 v{s_acc_lo[4 * q + d], (long long)s_acc_hi[4 * q + d]};
      acc128((unsigned long long*)&a.cell_geo[8 * (size_t)i + 2 * d], signed128(v, sd.sign));
      s_acc_lo[4 * q + d] = 0;
      s_acc_hi[4 * q + d] = 0;
    }
    s_acc_chi[q] = 0;
    s_acc_np[q] = 0;
  }
  if (!split || !next_chunk(sub, sub_n, single_end, ntb_all)) break;
  __syncthreads();  // the next chunk reuses every shared array
  }
  __syncthreads();  // the next item reuses every shared array
  if (a.item_cost && tid == 0)  // the item's duration (every thread is past it), a scheduling hint for the next build
    a.item_cost[item] = (unsigned)min(wall_clock64() - clock0, 0xffffffffull);
  }
  if (tid < 4) s_cnt[tid] = 0;
  __syncthreads();
  atomicAdd(&s_cnt[0], n_pairs);
  atomicAdd(&s_cnt[1], n64);
  __syncthreads();
  if (tid == 0 && n_cand) {
    if (s_cnt[0]) stat_add(a, C_PAIRS, s_cnt[0]);
    if (s_cnt[1]) stat_add(a, C_FP64, s_cnt[1]);
    stat_add(a, C_CAND, n_cand);
  }
}

// ---------------------------------------------------------------------------------------------------------------
// large-capacity kernel: one wavefront per deferred item, FP64 constructions, exact predicates, global scratch
// ---------------------------------------------------------------------------------------------------------------
struct SlowScratch {  // per wave, in global memory: the candidate lists, their vertex values, the global-memory polytopes
  static constexpr size_t cand_bytes = SLOW_KMAX * sizeof(int);
  static constexpr size_t key_bytes = SLOW_KMAX * sizeof(double);
  static constexpr size_t g_bytes = SLOW_KMAX * 4 * sizeof(double);   // g_j at the four tet vertices
  static constexpr size_t wave_bytes = 2 * (cand_bytes + key_bytes) + g_bytes;  // unsorted and sorted lists
  static constexpr size_t xyz_bytes = 64 * SLOW_VMAX * sizeof(Coord4<double>::type);  // [slot][lane]
  static constexpr size_t topo_bytes = 64 * SLOW_VMAX * sizeof(unsigned long long);    // [slot][lane]
  static constexpr size_t tab_bytes = 64 * (size_t)SLOW_PMAX;                          // [plane][lane]
  static constexpr size_t bytes = wave_bytes + xyz_bytes + topo_bytes + tab_bytes;
};
constexpr int SLOW_LDS_ITEMS = 512;  // the first deferred items go to the LDS variant (one item per wave)

// The LDS variant (few items: latency) keeps the candidate lists and 32 lanes' polytopes (32 vertices) in LDS; an item
// with more than 256 candidates, or a piece with more vertices, is handed to the global variant through the overflow
// list. The global variant (many items: throughput) keeps the lists and all 64 lanes' polytopes (64 vertices) in its
// scratch and takes the items past the LDS variant's share, then the overflow list.
template <bool LDS>
struct SlowCfg;
template <>
struct SlowCfg<true> {
  static constexpr int CL = 32, VCAP = 32, KCAP = 256;
  typedef unsigned Mask;
};
template <>
struct SlowCfg<false> {
  static constexpr int CL = 64, VCAP = SLOW_VMAX, KCAP = SLOW_KMAX;
  typedef unsigned long long Mask;
};

__device__ inline void push_overflow(const ShapeArgs& a, int4 item) {
  const unsigned long long idx = atomicAdd(&a.counters[C_DEFER2], 1ull);
  if (idx < (unsigned long long)a.deferred2_cap) a.deferred2[idx] = item;
  else atomicOr(a.status, ST_TABLE_FULL);
}

// One wavefront per deferred item: the lanes split the scan over all of the shape's sites (candidates are
// compacted in ascending site order by ballots), drop dominated candidates and rank-sort the rest, then clip the
// pieces with FP64 polytopes (lanes interleaved slot by slot).
template <bool LDS>
__global__ __launch_bounds__(64, LDS ? 1 : 2) void k_clip_slow(ShapeArgs a, unsigned char* scratch, int item_begin, int item_end) {
  typedef SlowCfg<LDS> C;
  constexpr int CL = C::CL, KC = C::KCAP;
  __shared__ Coord4<double>::type s_xyz[LDS ? C::VCAP * CL : 1];
  __shared__ unsigned long long s_topo[LDS ? C::VCAP * CL : 1];
  __shared__ unsigned char s_tab[LDS ? (4 + KC) * CL : 1];
  __shared__ int s_cand[LDS ? 2 * KC : 1];
  __shared__ double s_key[LDS ? 6 * KC : 1];
  // on-chip copies for the clipping loop, whose plane rebuilds would otherwise wait on memory: the item's tet and
  // the sites of its first SC candidates (sorted positions)
  constexpr int SC = 256;
  __shared__ float4 s_tv4[4];
  __shared__ double4 s_tf4[4];
  __shared__ float4 s_csite[SC];
  const int n_main = (int)min(min(a.counters[C_DEFER_ITEMS], (unsigned long long)a.deferred_cap),
                              (unsigned long long)item_end);
  const int n_over = LDS ? 0 : (int)min(a.counters[C_DEFER2], (unsigned long long)a.deferred2_cap);
  const int n_items = max(n_main - item_begin, 0) + n_over;
  const int lane = threadIdx.x;
  unsigned char* wbase = scratch + (size_t)blockIdx.x * SlowScratch::bytes;
  int* cand = LDS ? s_cand : (int*)wbase;
  int* scand = LDS ? s_cand + KC : (int*)(wbase + SlowScratch::cand_bytes + SlowScratch::key_bytes);
  double* key = LDS ? s_key : (double*)(wbase + SlowScratch::cand_bytes);
  double* skey = LDS ? s_key + KC : (double*)(wbase + 2 * SlowScratch::cand_bytes + SlowScratch::key_bytes);
  double* gv = LDS ? s_key + 2 * KC : (double*)(wbase + 2 * (SlowScratch::cand_bytes + SlowScratch::key_bytes));
  const int cl_lane = lane < CL ? lane : 0;
  Coord4<double>::type* xyz =
      LDS ? s_xyz + cl_lane : (Coord4<double>::type*)(wbase + SlowScratch::wave_bytes) + cl_lane;
  unsigned long long* topo =
      LDS ? s_topo + cl_lane
          : (unsigned long long*)(wbase + SlowScratch::wave_bytes + SlowScratch::xyz_bytes) + cl_lane;
  unsigned char* tab =
      LDS ? s_tab + cl_lane : wbase + SlowScratch::wave_bytes + SlowScratch::xyz_bytes + SlowScratch::topo_bytes + cl_lane;
  unsigned long long n_pairs = 0, n64 = 0, nex = 0;
  for (int vi = blockIdx.x; vi < n_items; vi += gridDim.x) {
    const int main_count = max(n_main - item_begin, 0);
    const int4 di = vi < main_count ? a.deferred[item_begin + vi] : a.deferred2[vi - main_count];
    const ShapeDesc sd = a.shapes[__builtin_amdgcn_readfirstlane(di.x)];
    const int t = di.y;
    const int want = di.z;
    const float4* ssite = a.site + sd.site_off;
    float4 tv[4];
    for (int v = 0; v < 4; ++v) tv[v] = sd.tp[4 * (size_t)t + v];
    if (lane < 4) {
      s_tv4[lane] = sd.tp[4 * (size_t)t + lane];
      s_tf4[lane] = sd.tf[4 * (size_t)t + lane];
    }
    const float4 o = tv[0];
    double y[3][3];
    for (int v = 1; v < 4; ++v) {
      y[v - 1][0] = (double)tv[v].x - o.x;
      y[v - 1][1] = (double)tv[v].y - o.y;
      y[v - 1][2] = (double)tv[v].z - o.z;
    }
    const double ycx = (y[0][0] + y[1][0] + y[2][0]) * 0.25, ycy = (y[0][1] + y[1][1] + y[2][1]) * 0.25,
                 ycz = (y[0][2] + y[1][2] + y[2][2]) * 0.25;
    // the fast kernel hands over the sorted candidates of the tets and pieces it defers when they fit its list (a
    // function of the tet's candidates only); otherwise they are found here among all sites
    const int m_list = di.w & 63;
    int m = 0;
    if (m_list > 0) {
      const int* lst = a.deferred_list + (size_t)(di.w >> 6) * KRAW;
      for (int x = lane; x < m_list; x += 64) {
        const int sx = lst[x];
        scand[x] = sx;
        if (x < SC) s_csite[x] = a.site[sx];
      }
      m = m_list;
      __syncthreads();
    } else {
      // candidates among ALL sites of the shape (same exact test as the fast kernel)
      double U = INFINITY;
      for (int j = lane; j < sd.ns; j += 64) {
        float4 s = ssite[j];
        double ax_ = (double)s.x - o.x, ay_ = (double)s.y - o.y, az_ = (double)s.z - o.z;
        double D = ax_ * ax_ + ay_ * ay_ + az_ * az_ - (double)s.w * s.w;
        double gmx = D;
        for (int v = 0; v < 3; ++v) gmx = fmax(gmx, D - 2.0 * (y[v][0] * ax_ + y[v][1] * ay_ + y[v][2] * az_));
        U = fmin(U, gmx);
      }
      for (int off = 32; off > 0; off >>= 1) U = fmin(U, __shfl_xor(U, off));
      if (a.tet_U && sd.sign > 0 && lane == 0) a.tet_U[sd.tet_off + t] = U;
      for (int base = 0; base < sd.ns; base += 64) {
        const int j = base + lane;
        bool take = false;
        double kk = 0.0;
        if (j < sd.ns) {
          float4 s = ssite[j];
          double ax_ = (double)s.x - o.x, ay_ = (double)s.y - o.y, az_ = (double)s.z - o.z;
          double D = ax_ * ax_ + ay_ * ay_ + az_ * az_ - (double)s.w * s.w;
          double gmn = D;
          for (int v = 0; v < 3; ++v) gmn = fmin(gmn, D - 2.0 * (y[v][0] * ax_ + y[v][1] * ay_ + y[v][2] * az_));
          take = gmn <= U;
          kk = D - 2.0 * (ycx * ax_ + ycy * ay_ + ycz * az_);
        }
        unsigned long long mask = __ballot(take);
        int pos = m + __popcll(mask & ((1ull << lane) - 1ull));
        if (take && pos < KC) {
          cand[pos] = sd.site_off + j;
          key[pos] = kk;
        }
        m += __popcll(mask);
      }
      if (m > KC) {
        if (lane == 0) {
          if (LDS) push_overflow(a, di);
          else atomicOr(a.status, ST_SLOW_CAPACITY);
        }
        continue;
      }
      __syncthreads();
      // drop every candidate that another one beats at all four tet vertices (g is affine, so then everywhere on the
      // tet: it owns nothing and its bisector constrains no piece); the values are exact in FP64
      for (int x = lane; x < m; x += 64) {
        const float4 s = a.site[cand[x]];
        const double ax_ = (double)s.x - o.x, ay_ = (double)s.y - o.y, az_ = (double)s.z - o.z;
        const double D = ax_ * ax_ + ay_ * ay_ + az_ * az_ - (double)s.w * s.w;
        gv[4 * x] = D;
        for (int v = 0; v < 3; ++v) gv[4 * x + 1 + v] = D - 2.0 * (y[v][0] * ax_ + y[v][1] * ay_ + y[v][2] * az_);
      }
      __syncthreads();
      int kept = 0;
      for (int base = 0; base < m; base += 64) {
        const int x = base + lane;
        bool keep = false;
        double kx = 0.0;
        int cx = 0;
        if (x < m) {
          const double g0 = gv[4 * x], g1 = gv[4 * x + 1], g2 = gv[4 * x + 2], g3 = gv[4 * x + 3];
          keep = true;
          for (int q = 0; q < m && keep; ++q)
            keep = !(gv[4 * q] < g0 && gv[4 * q + 1] < g1 && gv[4 * q + 2] < g2 && gv[4 * q + 3] < g3);
          kx = key[x];
          cx = cand[x];
        }
        const unsigned long long mask = __ballot(keep);
        __syncthreads();  // every lane has read cand/key of this chunk before they are overwritten in place
        if (keep) {
          const int pos = kept + __popcll(mask & ((1ull << lane) - 1ull));
          cand[pos] = cx;
          key[pos] = kx;
        }
        kept += __popcll(mask);
      }
      m = kept;
      __syncthreads();
      // rank sort by (key, position): positions ascend with the site id, so ties keep the site order
      for (int x = lane; x < m; x += 64) {
        const double kx = key[x];
        int rank = 0;
        for (int q = 0; q < m; ++q) {
          const double kq = key[q];
          rank += (kq < kx || (kq == kx && q < x)) ? 1 : 0;
        }
        scand[rank] = cand[x];
        skey[rank] = kx;
        if (rank < SC) s_csite[rank] = a.site[cand[x]];
      }
    }
    if (lane < CL)
      for (int k = 0; k < 4 + m; ++k) tab[CL * k] = 0;  // the plane ids of this item start unpaired
    __syncthreads();
    for (int ci = lane; ci < m && lane < CL; ci += CL) {
      if (want >= 0 && scand[ci] != want) continue;
      Clipper<double, Topo64, typename C::Mask, C::VCAP, true, MemTab> cl;
      cl.st.c = xyz;
      cl.st.w = topo;
      cl.st.stride = CL;
      cl.tab = MemTab{tab, CL};
      cl.a = &a;
      cl.flags = a.flags & ~RPD_FORCE_FP64;
      cl.np = 4 + m;
      cl.n64 = 0;
      cl.nex = 0;
      cl.env.tv = s_tv4;
      cl.env.o = s_tv4[0];
      cl.env.face64 = s_tf4;
      cl.env.sites = a.site;
      cl.env.sid = nullptr;  // candidates hold batch-global site ids directly
      cl.env.cidx8 = nullptr;
      cl.env.cidx32 = scand;
      cl.env.csite = s_csite;
      cl.env.ncs = min(m, SC);
      cl.env.ci = ci;
      cl.env.si = a.site[scand[ci]];
      cl.env.site_i = scand[ci];
      int r = clip_piece(cl, m, a.status);
      n64 += cl.n64;
      nex += cl.nex;
      if (r == CLIP_FULL) {  // out of vertex slots: the global variant redoes the piece with the same candidates
        if (LDS) push_overflow(a, make_int4(di.x, t, scand[ci], di.w));
        else atomicOr(a.status, ST_SLOW_CAPACITY);
        continue;
      }
      if (r == CLIP_OK) {
        n_pairs += (unsigned long long)(long long)sd.sign;
        emit_piece(cl, sd, t, a, CellSink{nullptr, nullptr, nullptr, nullptr, 0, -1});
      }
    }
    __syncthreads();  // the candidate list is rewritten by the next item
  }
  for (int off = 32; off > 0; off >>= 1) {
    n_pairs += __shfl_xor(n_pairs, off);
    n64 += __shfl_xor(n64, off);
    nex += __shfl_xor(nex, off);
  }
  if (lane == 0) {
    if (n_pairs) stat_add(a, C_PAIRS, n_pairs);
    if (n64) stat_add(a, C_FP64, n64);
    if (nex) stat_add(a, C_EXACT, nex);
  }
}

// ---------------------------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------------------------
template <typename T, int NT, int SLOTS>
static hipError_t launch_items(const ShapeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_clip_fast<T, NT, SLOTS>), dim3(a.nitems), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_clip_fast(const ShapeArgs& a, int precision, int block, int slots, hipStream_t s) {
  if (a.nitems == 0) return hipSuccess;
  if (precision == RPD_FP64) return launch_items<double, 64, 16>(a, s);
  if (block == 128) return launch_items<float, 128, 16>(a, s);
  if (block == 256) return launch_items<float, 256, 16>(a, s);
  if (slots == 12) return launch_items<float, 64, 12>(a, s);  // eight workgroups per compute unit
  return launch_items<float, 64, 16>(a, s);  // 64 threads (also for block 0): six workgroups per compute unit
}

size_t slow_scratch_bytes(int waves) { return (size_t)waves * SlowScratch::bytes; }

// the first SLOW_LDS_ITEMS items by the LDS variant, the rest by the global one (whose waves exit at once when there
// is no rest); the item count is read on the device
hipError_t launch_clip_slow(const ShapeArgs& a, unsigned char* scratch, int waves, hipStream_t s) {
  const int lds_waves = waves < SLOW_LDS_ITEMS ? waves : SLOW_LDS_ITEMS;
  hipLaunchKernelGGL(k_clip_slow<true>, dim3(lds_waves), dim3(64), 0, s, a, scratch, 0, SLOW_LDS_ITEMS);
  hipLaunchKernelGGL(k_clip_slow<false>, dim3(waves), dim3(64), 0, s, a, scratch, SLOW_LDS_ITEMS, INT_MAX);
  return hipGetLastError();
}

}  // namespace rpd
