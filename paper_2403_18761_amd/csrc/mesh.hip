// Mesh preprocessing (paper Sec. 4.1.2: the fractional weights are derived from the combinatorial structure of the
// tet mesh and shipped with it to the GPU). On the device: validation, a Morton ordering of the tets (so that a
// workgroup's tets are spatially compact), face adjacency and the multiplicity k(sigma) of every vertex, edge and
// face through hash tables, the weight numerators L/k(sigma) per tet, the component count and V - E + F - C.
#include <cstring>

#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include <cmath>
#include <numeric>
#include <vector>

#include "rpd_device.h"
#include "rpd_host.h"
#include "rpd_launch.h"

namespace rpd {

constexpr int KPRES = 4096;  // multiplicities k(sigma) must stay below this

enum { MS_INVALID = 1, MS_MESH = 2, MS_TOO_MANY_VERTS = 4, MS_TABLE = 8, MS_EDGE_LINK = 16, MS_VERT_LINK = 32 };

__device__ inline bool grid_ok(float v) {
  if (!(fabsf(v) <= 1.0f)) return false;
  float s = v * 1048576.0f;
  return s == rintf(s);
}

__global__ void k_mesh_verts(const float* vx, const float* vy, const float* vz, int nv, int* st) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x)
    if (!grid_ok(vx[v]) || !grid_ok(vy[v]) || !grid_ok(vz[v])) atomicOr(st, MS_INVALID);
}

__device__ inline unsigned long long spread3(unsigned long long x) {  // 21 bits -> every third bit
  x &= 0x1fffff;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__global__ void k_mesh_tets(const int* tv, int nt, int nv, const float* vx, const float* vy, const float* vz, int* st,
                            unsigned long long* mkey, int* idx) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x) {
    int q[4];
    bool ok = true;
    for (int k = 0; k < 4; ++k) {
      q[k] = tv[4 * (size_t)t + k];
      if (q[k] < 0 || q[k] >= nv) ok = false;
    }
    idx[t] = t;
    if (!ok) {
      atomicOr(st, MS_INVALID);
      mkey[t] = 0;
      continue;
    }
    long long X[4], Y[4], Z[4];
    for (int k = 0; k < 4; ++k) {
      X[k] = grid_int(vx[q[k]]);
      Y[k] = grid_int(vy[q[k]]);
      Z[k] = grid_int(vz[q[k]]);
    }
    long long ax = X[1] - X[0], ay = Y[1] - Y[0], az = Z[1] - Z[0];
    long long bx = X[2] - X[0], by = Y[2] - Y[0], bz = Z[2] - Z[0];
    long long cx = X[3] - X[0], cy = Y[3] - Y[0], cz = Z[3] - Z[0];
    i128 det = (i128)ax * ((i128)by * cz - (i128)bz * cy) - (i128)ay * ((i128)bx * cz - (i128)bz * cx) +
               (i128)az * ((i128)bx * cy - (i128)by * cx);
    if (det <= 0) atomicOr(st, MS_INVALID);
    long long sx = X[0] + X[1] + X[2] + X[3] + (1ll << 22), sy = Y[0] + Y[1] + Y[2] + Y[3] + (1ll << 22),
              sz = Z[0] + Z[1] + Z[2] + Z[3] + (1ll << 22);
    unsigned long long ux = (unsigned long long)min(sx >> 2, (1ll << 21) - 1);
    unsigned long long uy = (unsigned long long)min(sy >> 2, (1ll << 21) - 1);
    unsigned long long uz = (unsigned long long)min(sz >> 2, (1ll << 21) - 1);
    mkey[t] = (spread3(ux) << 2) | (spread3(uy) << 1) | spread3(uz);
  }
}

__global__ void k_mesh_gather(const int* tv, const int* perm, int nt, int nv, const float* vx, const float* vy,
                              const float* vz, float4* tp, int* itv, int* kv) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
    int o = perm[k];
    for (int v = 0; v < 4; ++v) {
      int q = tv[4 * (size_t)o + v];
      if (q < 0 || q >= nv) q = 0;  // already reported as invalid; keep every access in bounds
      tp[4 * (size_t)k + v] = make_float4(vx[q], vy[q], vz[q], 0.0f);
      itv[4 * (size_t)k + v] = q;
      atomicAdd(&kv[q], 1);
    }
  }
}

// the four face planes of every tet in FP64 (tet-local frame), computed once per mesh: the exact integer plane with its
// offset rounded once, which every FP64 filter reads instead of rebuilding it with 128-bit products
__global__ void k_mesh_faces64(const float4* tp, int nt, double4* tf) {
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < 4ll * nt; q += (long long)gridDim.x * blockDim.x) {
    const Plane<double> P = face_plane64(tp + 4 * (q >> 2), (int)(q & 3));
    tf[q] = make_double4(P.nx, P.ny, P.nz, P.d);
  }
}

__global__ void k_mesh_simplices(const int* itv, int nt, HashTab Eh, HashTab Fh, int* tedge, int* tface, int* ke,
                                 int* kf, int* face_t, int* st) {
  const int EV[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
    int q[4];
    for (int v = 0; v < 4; ++v) q[v] = itv[4 * (size_t)k + v];
    for (int e = 0; e < 6; ++e) {
      unsigned a = (unsigned)q[EV[e][0]], b = (unsigned)q[EV[e][1]];
      if (a == b) atomicOr(st, MS_INVALID);
      unsigned long long key = ((unsigned long long)min(a, b) << 32) | max(a, b);
      int s = ht_insert(Eh, key, st);
      if (s < 0) {
        atomicOr(st, MS_TABLE);
        continue;
      }
      tedge[6 * (size_t)k + e] = s;
      atomicAdd(&ke[s], 1);
    }
    for (int f = 0; f < 4; ++f) {
      unsigned w[3];
      int c = 0;
      for (int v = 0; v < 4; ++v)
        if (v != f) w[c++] = (unsigned)q[v];
      if (w[0] > w[1]) { unsigned x = w[0]; w[0] = w[1]; w[1] = x; }
      if (w[1] > w[2]) { unsigned x = w[1]; w[1] = w[2]; w[2] = x; }
      if (w[0] > w[1]) { unsigned x = w[0]; w[0] = w[1]; w[1] = x; }
      unsigned long long key = ((unsigned long long)w[0] << 42) | ((unsigned long long)w[1] << 21) | w[2];
      int s = ht_insert(Fh, key, st);
      if (s < 0) {
        atomicOr(st, MS_TABLE);
        continue;
      }
      tface[4 * (size_t)k + f] = s;
      int n = atomicAdd(&kf[s], 1);
      if (n < 2) face_t[2 * (size_t)s + n] = k;
      else atomicOr(st, MS_MESH);
    }
  }
}

__global__ void k_mesh_neighbours(const int* tface, const int* face_t, const int* kf, int nt, int* tn) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
    for (int f = 0; f < 4; ++f) {
      int s = tface[4 * (size_t)k + f];
      int nb = -1;
      if (kf[s] == 2) nb = face_t[2 * (size_t)s] == k ? face_t[2 * (size_t)s + 1] : face_t[2 * (size_t)s];
      tn[4 * (size_t)k + f] = nb;
    }
  }
}

// Manifold links (Sec. 3.3, Assumption: the input is a manifold tet mesh), by counting over the face and edge tables.
// Edge e: the tets around e, joined through the faces that contain e, form chains; a chain of m tets has m - 1
// shared faces when open (its two end faces lie on the boundary) and m when closed, so e has one chain exactly when
// (shared faces = k_e, no boundary face) or (shared faces = k_e - 1, two boundary faces). (Two closed chains around
// one edge would overlap in space, which the tets of a solid cannot.) Vertex v: the link surface, one vertex per edge
// at v, one edge per face at v and one triangle per tet at v, must be a sphere (V - E + F = 2, no boundary face at v)
// or a disk (1, with boundary faces); a pinched vertex, whose link falls apart into several spheres or disks, has a
// larger characteristic.
__global__ void k_link_faces(HashTab Fh, const int* kf, HashTab Eh, int* vf, int* vb, int* eint, int* ebnd) {
  const unsigned cap = Fh.mask + 1;
  for (unsigned s = blockIdx.x * blockDim.x + threadIdx.x; s < cap; s += gridDim.x * blockDim.x) {
    const unsigned long long key = Fh.keys[s];
    if (key == EMPTY_KEY) continue;
    const unsigned w[3] = {(unsigned)(key >> 42), (unsigned)((key >> 21) & 0x1fffff), (unsigned)(key & 0x1fffff)};
    const bool bnd = kf[s] == 1;
    for (int k = 0; k < 3; ++k) {
      atomicAdd(&vf[w[k]], 1);
      if (bnd) atomicAdd(&vb[w[k]], 1);
    }
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
    for (int k = 0; k < 3; ++k) {  // w is ascending, so every pair is an edge key (min << 32 | max)
      const int e = ht_find(Eh, ((unsigned long long)w[pa[k]] << 32) | w[pb[k]]);
      if (e >= 0) atomicAdd(bnd ? &ebnd[e] : &eint[e], 1);
    }
  }
}
__global__ void k_link_edges(HashTab Eh, const int* ke, const int* eint, const int* ebnd, int* ve, int* st) {
  const unsigned cap = Eh.mask + 1;
  for (unsigned s = blockIdx.x * blockDim.x + threadIdx.x; s < cap; s += gridDim.x * blockDim.x) {
    const unsigned long long key = Eh.keys[s];
    if (key == EMPTY_KEY) continue;
    atomicAdd(&ve[(unsigned)(key >> 32)], 1);
    atomicAdd(&ve[(unsigned)(key & 0xffffffffull)], 1);
    const int k = ke[s], fi = eint[s], fb = ebnd[s];
    if (!((fi == k && fb == 0) || (fi == k - 1 && fb == 2))) atomicOr(st, MS_EDGE_LINK);
  }
}
__global__ void k_link_verts(const int* kv, const int* ve, const int* vf, const int* vb, int nv, int* st) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    if (kv[v] == 0) continue;
    const int chi = ve[v] - vf[v] + kv[v];
    if (!((chi == 2 && vb[v] == 0) || (chi == 1 && vb[v] > 0))) atomicOr(st, MS_VERT_LINK);
  }
}

__global__ void k_presence(const int* kcount, int n, int* pres, int* used, int* st) {
  int local = 0;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    int k = kcount[s];
    if (k <= 0) continue;
    ++local;
    if (k >= KPRES) atomicOr(st, MS_MESH);
    else pres[k] = 1;
  }
  if (local) atomicAdd(used, local);
}

// owner of every vertex, edge and face: the lowest caller tet index among the tets containing it
__global__ void k_owners(const int* itv, const int* tedge, const int* tface, const int* perm, int nt, int* ov,
                         int* oe, int* of) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
    const int c = perm[k];
    for (int v = 0; v < 4; ++v) atomicMin(&ov[itv[4 * (size_t)k + v]], c);
    for (int e = 0; e < 6; ++e) atomicMin(&oe[tedge[6 * (size_t)k + e]], c);
    for (int f = 0; f < 4; ++f) atomicMin(&of[tface[4 * (size_t)k + f]], c);
  }
}

// weight numerators of a tet's 4 vertices, 6 edges and 4 faces: L / k(sigma), or with owners (ov != nullptr)
// 1 in the owner tet and 0 elsewhere
__global__ void k_weights(const int* itv, const int* tedge, const int* tface, const int* kv, const int* ke,
                          const int* kf, int nt, long long L, const int* perm, const int* ov, const int* oe,
                          const int* of, unsigned* nu, unsigned long long* vol, const float4* tp) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
    unsigned* o = nu + 14 * (size_t)k;
    if (ov) {
      const int c = perm[k];
      for (int v = 0; v < 4; ++v) o[v] = ov[itv[4 * (size_t)k + v]] == c;
      for (int e = 0; e < 6; ++e) o[4 + e] = oe[tedge[6 * (size_t)k + e]] == c;
      for (int f = 0; f < 4; ++f) o[10 + f] = of[tface[4 * (size_t)k + f]] == c;
    } else {
      for (int v = 0; v < 4; ++v) o[v] = (unsigned)(L / kv[itv[4 * (size_t)k + v]]);
      for (int e = 0; e < 6; ++e) o[4 + e] = (unsigned)(L / ke[tedge[6 * (size_t)k + e]]);
      for (int f = 0; f < 4; ++f) o[10 + f] = (unsigned)(L / kf[tface[4 * (size_t)k + f]]);
    }
    const float4* p = tp + 4 * (size_t)k;
    double ax = (double)p[1].x - p[0].x, ay = (double)p[1].y - p[0].y, az = (double)p[1].z - p[0].z;
    double bx = (double)p[2].x - p[0].x, by = (double)p[2].y - p[0].y, bz = (double)p[2].z - p[0].z;
    double cx = (double)p[3].x - p[0].x, cy = (double)p[3].y - p[0].y, cz = (double)p[3].z - p[0].z;
    double det = ax * (by * cz - bz * cy) - ay * (bx * cz - bz * cx) + az * (bx * cy - by * cx);
    atomicAdd(vol, (unsigned long long)llrint(det / 6.0 * 72057594037927936.0));
  }
}

__device__ inline int uf_find_m(int* par, int x) {
  while (true) {
    int p = par[x];
    if (p == x) return x;
    int gp = par[p];
    if (gp != p) par[x] = gp;
    x = p;
  }
}
__global__ void k_tet_uf_init(int* par, int nt) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) par[k] = k;
}
__global__ void k_tet_uf(const int* tn, int nt, int* par) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
    for (int f = 0; f < 4; ++f) {
      int b = tn[4 * (size_t)k + f];
      if (b < 0 || b < k) continue;
      int x = k, y = b;
      while (true) {
        x = uf_find_m(par, x);
        y = uf_find_m(par, y);
        if (x == y) break;
        if (x < y) { int t = x; x = y; y = t; }
        if (atomicCAS(&par[x], x, y) == x) break;
      }
    }
  }
}
__global__ void k_tet_roots(int* par, int nt, int* roots) {
  int local = 0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x)
    if (uf_find_m(par, k) == k) ++local;
  if (local) atomicAdd(roots, local);
}

static int gsz(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return (int)(g ? g : 1);
}

static unsigned pow2_at_least(size_t n) {
  size_t c = 1024;
  while (c < n) c <<= 1;
  return (unsigned)c;
}

static long long gcdll(long long a, long long b) {
  while (b) {
    long long t = a % b;
    a = b;
    b = t;
  }
  return a;
}

void mesh_prepare(rpd_mesh* m, const rpd_mesh_desc* d, uint32_t flags, hipStream_t s) {
  const int nv = d->n_verts, nt = d->n_tets;
  if (nv <= 0 || nt <= 0 || !d->vx || !d->vy || !d->vz || !d->tv) throw Failure{RPD_E_INVALID, "empty mesh"};
  if (nv >= (1 << 21)) throw Failure{RPD_E_INVALID, "more than 2^21 - 1 vertices"};
  if (nt >= (1 << 30)) throw Failure{RPD_E_INVALID, "more than 2^30 tets"};
  m->nv = nv;
  m->nt = nt;
  const bool dev = (flags & RPD_DEVICE_PTRS) != 0;
  DBuf vx, vy, vz, tv;
  const float *pvx = d->vx, *pvy = d->vy, *pvz = d->vz;
  const int* ptv = d->tv;
  if (!dev) {
    vx.alloc(sizeof(float) * nv);
    vy.alloc(sizeof(float) * nv);
    vz.alloc(sizeof(float) * nv);
    tv.alloc(sizeof(int) * 4 * (size_t)nt);
    hip_check(hipMemcpyAsync(vx.p, d->vx, sizeof(float) * nv, hipMemcpyHostToDevice, s), "upload");
    hip_check(hipMemcpyAsync(vy.p, d->vy, sizeof(float) * nv, hipMemcpyHostToDevice, s), "upload");
    hip_check(hipMemcpyAsync(vz.p, d->vz, sizeof(float) * nv, hipMemcpyHostToDevice, s), "upload");
    hip_check(hipMemcpyAsync(tv.p, d->tv, sizeof(int) * 4 * (size_t)nt, hipMemcpyHostToDevice, s), "upload");
    pvx = vx.as<float>();
    pvy = vy.as<float>();
    pvz = vz.as<float>();
    ptv = tv.as<int>();
  }
  DBuf st(sizeof(int) * 8);
  hip_check(hipMemsetAsync(st.p, 0, sizeof(int) * 8, s), "memset");
  int* pst = st.as<int>();
  hipLaunchKernelGGL(k_mesh_verts, dim3(gsz(nv)), dim3(256), 0, s, pvx, pvy, pvz, nv, pst);
  // Morton order of the tet centroids
  DBuf mkey(sizeof(unsigned long long) * nt), mkey2(sizeof(unsigned long long) * nt), idx(sizeof(int) * nt);
  m->perm.alloc(sizeof(int) * nt);
  hipLaunchKernelGGL(k_mesh_tets, dim3(gsz(nt)), dim3(256), 0, s, ptv, nt, nv, pvx, pvy, pvz, pst,
                     mkey.as<unsigned long long>(), idx.as<int>());
  size_t tmpb = 0;
  hip_check(rocprim::radix_sort_pairs(nullptr, tmpb, mkey.as<unsigned long long>(), mkey2.as<unsigned long long>(),
                                      idx.as<int>(), m->perm.as<int>(), (size_t)nt, 0, 64, s),
            "sort");
  DBuf tmp(tmpb);
  hip_check(rocprim::radix_sort_pairs(tmp.p, tmpb, mkey.as<unsigned long long>(), mkey2.as<unsigned long long>(),
                                      idx.as<int>(), m->perm.as<int>(), (size_t)nt, 0, 64, s),
            "sort");
  // gather per-tet vertex data in internal order; vertex multiplicities
  m->tp.alloc(sizeof(float4) * 4 * (size_t)nt);
  DBuf itv(sizeof(int) * 4 * (size_t)nt), kv(sizeof(int) * nv);
  hip_check(hipMemsetAsync(kv.p, 0, sizeof(int) * nv, s), "memset");
  hipLaunchKernelGGL(k_mesh_gather, dim3(gsz(nt)), dim3(256), 0, s, ptv, m->perm.as<int>(), nt, nv, pvx, pvy, pvz,
                     m->tp.as<float4>(), itv.as<int>(), kv.as<int>());
  m->tf.alloc(sizeof(double4) * 4 * (size_t)nt);
  hipLaunchKernelGGL(k_mesh_faces64, dim3(gsz(4ll * nt)), dim3(256), 0, s, m->tp.as<float4>(), nt,
                     m->tf.as<double4>());
  // edges and faces
  // capacities at least the number of possible distinct keys (6 edges and 4 faces per tet): inserts cannot fail
  unsigned ecap = pow2_at_least(6 * (size_t)nt + 1024), fcap = pow2_at_least(4 * (size_t)nt + 1024);
  DBuf ekeys(sizeof(unsigned long long) * ecap), fkeys(sizeof(unsigned long long) * fcap);
  hip_check(launch_fill_u64(ekeys.as<unsigned long long>(), EMPTY_KEY, ecap, s), "fill");
  hip_check(launch_fill_u64(fkeys.as<unsigned long long>(), EMPTY_KEY, fcap, s), "fill");
  DBuf tedge(sizeof(int) * 6 * (size_t)nt), tface(sizeof(int) * 4 * (size_t)nt);
  DBuf ke(sizeof(int) * ecap), kf(sizeof(int) * fcap), face_t(sizeof(int) * 2 * (size_t)fcap);
  hip_check(hipMemsetAsync(ke.p, 0, sizeof(int) * ecap, s), "memset");
  hip_check(hipMemsetAsync(kf.p, 0, sizeof(int) * fcap, s), "memset");
  HashTab Eh{ekeys.as<unsigned long long>(), ecap - 1}, Fh{fkeys.as<unsigned long long>(), fcap - 1};
  hipLaunchKernelGGL(k_mesh_simplices, dim3(gsz(nt)), dim3(256), 0, s, itv.as<int>(), nt, Eh, Fh, tedge.as<int>(),
                     tface.as<int>(), ke.as<int>(), kf.as<int>(), face_t.as<int>(), pst);
  {  // edge and vertex links
    DBuf lnk(sizeof(int) * (3 * (size_t)nv + 2 * (size_t)ecap));
    hip_check(hipMemsetAsync(lnk.p, 0, lnk.bytes, s), "memset");
    int* vf = lnk.as<int>();
    int* vb = vf + nv;
    int* ve = vb + nv;
    int* eint = ve + nv;
    int* ebnd = eint + ecap;
    hipLaunchKernelGGL(k_link_faces, dim3(gsz(fcap)), dim3(256), 0, s, Fh, kf.as<int>(), Eh, vf, vb, eint, ebnd);
    hipLaunchKernelGGL(k_link_edges, dim3(gsz(ecap)), dim3(256), 0, s, Eh, ke.as<int>(), eint, ebnd, ve, pst);
    hipLaunchKernelGGL(k_link_verts, dim3(gsz(nv)), dim3(256), 0, s, kv.as<int>(), ve, vf, vb, nv, pst);
    hip_check(hipStreamSynchronize(s), "sync");  // the counters are released next
  }
  m->tn.alloc(sizeof(int) * 4 * (size_t)nt);
  hipLaunchKernelGGL(k_mesh_neighbours, dim3(gsz(nt)), dim3(256), 0, s, tface.as<int>(), face_t.as<int>(),
                     kf.as<int>(), nt, m->tn.as<int>());
  // multiplicities present -> L
  DBuf pres(sizeof(int) * (KPRES + 8));
  hip_check(hipMemsetAsync(pres.p, 0, sizeof(int) * (KPRES + 8), s), "memset");
  int* pp = pres.as<int>();
  hipLaunchKernelGGL(k_presence, dim3(gsz(nv)), dim3(256), 0, s, kv.as<int>(), nv, pp, pp + KPRES, pst);
  hipLaunchKernelGGL(k_presence, dim3(gsz(ecap)), dim3(256), 0, s, ke.as<int>(), (int)ecap, pp, pp + KPRES + 1, pst);
  hipLaunchKernelGGL(k_presence, dim3(gsz(fcap)), dim3(256), 0, s, kf.as<int>(), (int)fcap, pp, pp + KPRES + 2, pst);
  // components
  DBuf par(sizeof(int) * nt);
  hipLaunchKernelGGL(k_tet_uf_init, dim3(gsz(nt)), dim3(256), 0, s, par.as<int>(), nt);
  hipLaunchKernelGGL(k_tet_uf, dim3(gsz(nt)), dim3(256), 0, s, m->tn.as<int>(), nt, par.as<int>());
  hipLaunchKernelGGL(k_tet_roots, dim3(gsz(nt)), dim3(256), 0, s, par.as<int>(), nt, pp + KPRES + 3);
  hip_check(hipGetLastError(), "mesh kernels");
  std::vector<int> hp(KPRES + 8);
  int hst[8];
  hip_check(hipMemcpyAsync(hp.data(), pp, sizeof(int) * (KPRES + 8), hipMemcpyDeviceToHost, s), "download");
  hip_check(hipMemcpyAsync(hst, pst, sizeof(int) * 8, hipMemcpyDeviceToHost, s), "download");
  hip_check(hipStreamSynchronize(s), "sync");
  if (hst[0] & MS_INVALID) throw Failure{RPD_E_INVALID, "mesh: off-grid coordinate, bad index or non-positive tet"};
  if (hst[0] & MS_TABLE) throw Failure{RPD_E_INTERNAL, "mesh: hash table full"};
  if (hst[0] & MS_MESH) throw Failure{RPD_E_MESH, "mesh: a face is shared by more than two tets"};
  if (hst[0] & MS_EDGE_LINK) throw Failure{RPD_E_MESH, "mesh: non-manifold edge (its tets are not one chain)"};
  if (hst[0] & MS_VERT_LINK) throw Failure{RPD_E_MESH, "mesh: non-manifold vertex (its link is not a sphere or disk)"};
  long long L = 1;
  bool big = false;
  for (int k = 1; k < KPRES && !big; ++k)
    if (hp[k]) {
      L = L / gcdll(L, k) * k;
      big = L >= (1ll << 31);
    }
  m->owner = big || (flags & RPD_OWNER_WEIGHTS) ? 1 : 0;
  if (m->owner) L = 1;
  m->L = L;
  m->n_edges = hp[KPRES + 1];
  m->n_faces = hp[KPRES + 2];
  m->components = hp[KPRES + 3];
  m->euler = hp[KPRES] - m->n_edges + m->n_faces - nt;
  if (m->components != 1) throw Failure{RPD_E_MESH, "mesh: more than one connected component"};
  m->nu.alloc(sizeof(unsigned) * 14 * (size_t)nt);
  DBuf vol(sizeof(unsigned long long)), own_v, own_e, own_f;
  hip_check(hipMemsetAsync(vol.p, 0, sizeof(unsigned long long), s), "memset");
  if (m->owner) {
    own_v.alloc(sizeof(int) * nv);
    own_e.alloc(sizeof(int) * ecap);
    own_f.alloc(sizeof(int) * fcap);
    hip_check(launch_fill_i32(own_v.as<int>(), INT32_MAX, nv, s), "fill");
    hip_check(launch_fill_i32(own_e.as<int>(), INT32_MAX, ecap, s), "fill");
    hip_check(launch_fill_i32(own_f.as<int>(), INT32_MAX, fcap, s), "fill");
    hipLaunchKernelGGL(k_owners, dim3(gsz(nt)), dim3(256), 0, s, itv.as<int>(), tedge.as<int>(), tface.as<int>(),
                       m->perm.as<int>(), nt, own_v.as<int>(), own_e.as<int>(), own_f.as<int>());
  }
  hipLaunchKernelGGL(k_weights, dim3(gsz(nt)), dim3(256), 0, s, itv.as<int>(), tedge.as<int>(), tface.as<int>(),
                     kv.as<int>(), ke.as<int>(), kf.as<int>(), nt, L, m->perm.as<int>(), own_v.as<int>(),
                     own_e.as<int>(), own_f.as<int>(), m->nu.as<unsigned>(), vol.as<unsigned long long>(),
                     m->tp.as<float4>());
  hip_check(hipGetLastError(), "mesh weights");
  long long hv = 0;
  hip_check(hipMemcpyAsync(&hv, vol.p, sizeof(long long), hipMemcpyDeviceToHost, s), "download");
  hip_check(hipStreamSynchronize(s), "sync");
  m->volume = (double)hv / 72057594037927936.0;
  // Workgroup blocks: runs of at most TB consecutive tets (Morton order) inside one octree cell whose side is about
  // twice the mean tet size, so that every block has a small bounding box (a plain cut every TB tets can straddle
  // the jumps of the Morton curve and produce boxes as large as the solid).
  {
    std::vector<unsigned long long> keys(nt);
    hip_check(hipMemcpyAsync(keys.data(), mkey2.p, sizeof(unsigned long long) * nt, hipMemcpyDeviceToHost, s),
              "download");
    hip_check(hipStreamSynchronize(s), "sync");
    double edge = std::cbrt(6.0 * m->volume / nt) * 1048576.0;  // mean tet size in 2^-20 units
    int level = 0;
    while (level < 20 && (double)(1ll << (level + 1)) <= 2.0 * edge) ++level;
    const int shift = 3 * (level + 1);
    std::vector<int> starts;
    starts.push_back(0);
    for (int k = 1; k < nt; ++k) {
      bool cut = (keys[k] >> shift) != (keys[k - 1] >> shift) || k - starts.back() >= TB;
      if (cut) starts.push_back(k);
    }
    starts.push_back(nt);
    m->nblk = (int)starts.size() - 1;
    m->hblk = starts;
    m->blk.alloc(sizeof(int) * starts.size());
    hip_check(hipMemcpyAsync(m->blk.p, starts.data(), sizeof(int) * starts.size(), hipMemcpyHostToDevice, s), "upload");
    hip_check(hipStreamSynchronize(s), "sync");
  }
  (void)hipGetDevice(&m->device);
}

}  // namespace rpd
