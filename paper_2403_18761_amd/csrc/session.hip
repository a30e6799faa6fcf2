// Incremental RPD update inside a topology-repair loop (paper Sec. 4: spheres are inserted where an element is not
// contractible, and the RPD is updated only for the cells related to the new spheres, Sec. 4 overview and Sec. 5.2).
//
// One round, all on the device with device-side counts (so the round is captured once as a HIP graph):
//   1. select up to M violating cells (nonempty, chi != 1 or beta0 > 1), lowest ids first;
//   2. for each, pick a tet among the cell's pieces (outside the component of its piece in its smallest tet when
//      beta0 > 1) and insert a sphere: either the caller's per-tet table entry of the tet with the largest
//      (hash(tet, round), tet), tets in the caller's numbering, or (Sec. 4.1.3: the furthest surface triangle of the
//      cell is the pin of sphere shrinking) the shrunk sphere of the surface face, among those the cell touches,
//      furthest from the cell's sphere centre;
//   3. mark the workgroup blocks whose tets a new sphere may own (the exact candidate test against the stored U_t);
//   4. remove the contributions of the dirty blocks computed with the old sites, add them back with the new sites
//      (every accumulator is an exactly invertible integer), and recompute beta0 of the live element pieces.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rpd_device.h"
#include "rpd_launch.h"

namespace rpd {


__global__ void k_round_begin(RoundState r) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *r.nsel = 0;
    *r.nitems = 0;
  }
}

// first M violating cells in ascending order (one workgroup, chunked ballot compaction)
__global__ __launch_bounds__(256) void k_select(RoundState r, const long long* cell_chi, const int* cell_np,
                                                const int* cell_b0) {
  __shared__ int s_count;
  __shared__ int s_warp[4];
  const int n = *r.ns_cur;
  const long long L = r.new_desc->L;
  if (threadIdx.x == 0) s_count = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 256) {
    const int i = base + threadIdx.x;
    const bool v = i < n && cell_np[i] > 0 && (cell_chi[i] != L || cell_b0[i] > 1);
    unsigned long long m = __ballot(v);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_warp[w] = __popcll(m);
    __syncthreads();
    int before = s_count;
    for (int q = 0; q < w; ++q) before += s_warp[q];
    int pos = before + __popcll(m & ((1ull << lane) - 1ull));
    if (v && pos < r.max_insert) {
      r.sel[pos] = i;
      r.selpos[i] = pos;
      r.best[pos] = 0ull;
      r.ref[pos] = ~0ull;
    }
    __syncthreads();
    if (threadIdx.x == 0) s_count += s_warp[0] + s_warp[1] + s_warp[2] + s_warp[3];
    __syncthreads();
    if (s_count >= r.max_insert) break;
  }
  if (threadIdx.x == 0) *r.nsel = min(s_count, r.max_insert);
}

__device__ inline int uf_root(const NodeRec* rec, int x) {
  while (true) {
    int p = rec[x].parent;
    if (p == x) return x;
    x = p;
  }
}

// The scans over the element-piece table reduce into LDS slots of the selected cells first (dynamic LDS of
// max_insert entries) and flush once per workgroup, on a grid of a few workgroups per compute unit.
constexpr int SCAN_BLOCKS = 1024;

// the piece of every selected cell in its smallest tet (caller's numbering, so that the rule does not depend on the
// internal tet order), packed with its internal tet id for the lookup of its node
__global__ __launch_bounds__(256) void k_ref_tet(NodeTab N, RoundState r) {
  extern __shared__ unsigned long long s_ref[];
  const int nsel = *r.nsel;
  for (int k = threadIdx.x; k < nsel; k += blockDim.x) s_ref[k] = ~0ull;
  __syncthreads();
  for (int b = blockIdx.x; b < r.cnseg; b += gridDim.x) {
    const int n = r.cseg[b];
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const unsigned long long key = N.rec[r.clist[(size_t)b * r.clen + j]].key;  // a live cell piece
      int cell = (int)((key >> 32) & 0x3fffffff);
      int k = r.selpos[cell];
      if (k < 0) continue;
      const unsigned t = (unsigned)(key & 0xffffffffull);
      atomicMin(&s_ref[k], ((unsigned long long)(unsigned)r.perm[t] << 32) | t);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nsel; k += blockDim.x)
    if (s_ref[k] != ~0ull) atomicMin(&r.ref[k], s_ref[k]);
}

__device__ inline unsigned mix_hash(unsigned long long x) {  // splitmix64 finaliser
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return (unsigned)((x ^ (x >> 31)) >> 32);
}

__global__ __launch_bounds__(256) void k_pick_tet(NodeTab N, const int* cell_b0, RoundState r, const float4* tp,
                                                  const float4* site) {
  extern __shared__ unsigned long long s_best[];
  const int nsel = *r.nsel;
  for (int k = threadIdx.x; k < nsel; k += blockDim.x) s_best[k] = 0ull;
  __syncthreads();
  const int round = *r.round;
  for (int j = threadIdx.x, b = blockIdx.x; b < r.cnseg;) {  // the live cell pieces, segment by segment
    if (j >= r.cseg[b]) {
      j = threadIdx.x;
      b += gridDim.x;
      continue;
    }
    const int s = r.clist[(size_t)b * r.clen + j];
    j += blockDim.x;
    const NodeRec nr = N.rec[s];
    const unsigned long long key = nr.key;
    int cell = (int)((key >> 32) & 0x3fffffff);
    int k = r.selpos[cell];
    if (k < 0) continue;
    int t = (int)(key & 0xffffffffull);
    const int tc = r.perm[t];  // caller's tet id: the table's index and the hash input
    const int bnd = node_bnd_bits(nr.st);
    if (r.mode ? bnd == 0 : r.tet_used[tc] != 0) continue;
    if (cell_b0[cell] > 1) {  // pick outside the component of the cell's piece in its smallest tet
      int rs = node_find(N, (key & ~0xffffffffull) | (unsigned)(r.ref[k] & 0xffffffffull));
      if (rs >= 0 && uf_root(N.rec, rs) == uf_root(N.rec, s)) continue;
    }
    if (r.mode) {  // surface faces of tet t that the piece touches: the one furthest from the cell's centre
      const float4 c = site[cell];
      const float4* v = tp + 4 * (size_t)t;
      for (int f = 0; f < 4; ++f) {
        const int slot = 4 * t + f;
        if (!(bnd & (1 << f)) || r.tet_used[slot]) continue;
        float gx = 0.f, gy = 0.f, gz = 0.f;
        for (int q = 0; q < 4; ++q)
          if (q != f) {
            gx += v[q].x;
            gy += v[q].y;
            gz += v[q].z;
          }
        gx = gx * (1.f / 3.f) - c.x;
        gy = gy * (1.f / 3.f) - c.y;
        gz = gz * (1.f / 3.f) - c.z;
        const float d = __builtin_sqrtf(gx * gx + gy * gy + gz * gz);  // >= 0: its bits order like the value
        atomicMax(&s_best[k], ((unsigned long long)__float_as_uint(d) << 32) | (unsigned)slot);
      }
      continue;
    }
    unsigned h = mix_hash(((unsigned long long)(unsigned)tc << 32) | (unsigned)round);
    atomicMax(&s_best[k], ((unsigned long long)h << 32) | (unsigned)tc);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nsel; k += blockDim.x)
    if (s_best[k]) atomicMax(&r.best[k], s_best[k]);
}

// Insertion in selection order (deterministic site ids): cell k inserts its tet's sphere unless a cell earlier in
// the order chose the same tet, the tet's sphere is in already, or the site capacity is reached. One workgroup.
__global__ __launch_bounds__(1024) void k_insert(RoundState r, float4* site) {
  __shared__ unsigned long long s_b[MAX_INSERT];
  __shared__ int s_wave[16];
  __shared__ int s_total;
  const int n0 = *r.ns_cur;
  const int nsel = *r.nsel;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < nsel; k += blockDim.x) s_b[k] = r.best[k];
  if (threadIdx.x == 0) s_total = 0;
  __syncthreads();
  for (int base = 0; base < nsel; base += 1024) {
    const int k = base + threadIdx.x;
    bool win = false;
    int t = -1;
    if (k < nsel) {
      const unsigned long long b = s_b[k];
      t = (int)(b & 0xffffffffull);
      win = b != 0ull && !r.tet_used[t];
      for (int q = 0; q < k && win; ++q) {
        const unsigned long long bq = s_b[q];
        win = !(bq != 0ull && (int)(bq & 0xffffffffull) == t);
      }
    }
    const unsigned long long m = __ballot(win);
    if (lane == 0) s_wave[w] = __popcll(m);
    __syncthreads();
    int before = s_total;
    for (int q = 0; q < w; ++q) before += s_wave[q];
    const int pos = n0 + before + __popcll(m & ((1ull << lane) - 1ull));
    if (win && pos < r.max_sites) site[pos] = r.table[t];
    __syncthreads();  // every thread has read tet_used before it changes
    if (win && pos < r.max_sites) r.tet_used[t] = 1;
    if (threadIdx.x == 0) {
      int c = 0;
      for (int q = 0; q < 16; ++q) c += s_wave[q];
      s_total += c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int n = min(n0 + s_total, r.max_sites);
    r.old_desc->ns = n0;
    r.new_desc->ns = n;
    *r.ins_total += n - n0;
  }
}

// a tet is dirty if one of the new spheres passes its exact candidate test against the stored U_t
__global__ void k_mark_dirty(RoundState r, const float4* tp, int nt, const float4* site, const double* tet_U) {
  const int n0 = r.old_desc->ns, n1 = r.new_desc->ns;
  if (n1 == n0) return;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x) {
    const float4* tv = tp + 4 * (size_t)t;
    const float4 o = tv[0];
    const double U = tet_U[t];
    bool dirty = false;
    for (int j = n0; j < n1 && !dirty; ++j) {
      float4 s = site[j];
      double ax = (double)s.x - o.x, ay = (double)s.y - o.y, az = (double)s.z - o.z;
      double D = ax * ax + ay * ay + az * az - (double)s.w * s.w;
      double gmn = D;
      for (int v = 1; v < 4; ++v)
        gmn = fmin(gmn, D - 2.0 * (((double)tv[v].x - o.x) * ax + ((double)tv[v].y - o.y) * ay +
                                   ((double)tv[v].z - o.z) * az));
      dirty = gmn <= U;
    }
    if (dirty) {
      const int b = r.tet_block[t];
      atomicOr(&r.dirty[b], 1ull << (t - r.blk[b]));
    }
  }
}

// dirty tets -> work items, then clear the masks. Every part of SPLIT_TETS tets that holds a dirty tet becomes two
// items with the mask of its dirty tets: in any other tet no new sphere owns a point, so none of its pieces change.
// Dirty tets cluster where spheres go in, which is where the sites are densest, and parts spread them over more
// workgroups. Any order gives the same sums (integers); the blocks are scanned heaviest first so that the items
// come out in about that order, which shortens the clipping kernel's tail.
__global__ void k_dirty_items(RoundState r, int nblk) {
  static_assert(SPLIT_TETS == 16 && TB <= 64, "16-bit part masks of a 64-bit block mask");
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nblk; k += gridDim.x * blockDim.x) {
    const int b = r.order[k];
    const unsigned long long mask = r.dirty[b];
    if (!mask) continue;
    r.dirty[b] = 0;
    int parts = 0;  // parts with a dirty tet
    for (int p = 0; p < TB / SPLIT_TETS; ++p) parts += ((mask >> (SPLIT_TETS * p)) & 0xffffull) ? 1 : 0;
    // room for the active lanes' parts: one atomic per wavefront, offsets by a prefix over the active lanes
    const unsigned long long active = __ballot(1);
    const int lane = (int)__lane_id(), leader = __ffsll((long long)active) - 1;
    int before = 0, sum = 0;
    for (int q = 0; q < 64; ++q) {
      const int pq = __shfl(parts, q);
      if ((active >> q) & 1ull) {
        sum += pq;
        if (q < lane) before += pq;
      }
    }
    int base = 0;
    if (lane == leader) {
      base = atomicAdd(r.nitems, 2 * sum) / 2;
      atomicAdd(r.dirty_total, __popcll(active));
    }
    base = __shfl(base, leader);
    int2* out = r.items + 2 * (size_t)(base + before);
    for (int p = 0; p < TB / SPLIT_TETS; ++p) {
      const unsigned pm = (unsigned)((mask >> (SPLIT_TETS * p)) & 0xffffull);
      if (!pm) continue;
      const int y = b | ((p + 1) << ITEM_PART_SHIFT);
      *out++ = make_int2((int)(pm << 16), y);      // taken out from the state before the insertions
      *out++ = make_int2((int)(pm << 16) | 1, y);  // added from the state after them
    }
  }
}

__global__ void k_round_end(RoundState r) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int nsel = *r.nsel;
  for (int k = 0; k < nsel; ++k) r.selpos[r.sel[k]] = -1;
  *r.ns_cur = r.new_desc->ns;
  *r.round += 1;
}

static int gsz(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return (int)(g ? g : 1);
}

// Surface faces of the mesh (faces without a neighbour tet), compacted in any order: the triangle, its centroid as
// the pin and its unit normal towards the tet's opposite vertex (inward), and the face's slot 4 t + f.
__global__ void k_surface_faces(const float4* tp, const int* tn, int nt, float* tri, float* pin, float* nrm, int* slot,
                                int* count) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < 4 * nt; q += gridDim.x * blockDim.x) {
    if (tn[q] >= 0) continue;
    const int t = q >> 2, f = q & 3;
    const float4* v = tp + 4 * (size_t)t;
    double P[3][3];
    int c = 0;
    for (int k = 0; k < 4; ++k)
      if (k != f) {
        P[c][0] = v[k].x;
        P[c][1] = v[k].y;
        P[c][2] = v[k].z;
        ++c;
      }
    const double ux = P[1][0] - P[0][0], uy = P[1][1] - P[0][1], uz = P[1][2] - P[0][2];
    const double wx = P[2][0] - P[0][0], wy = P[2][1] - P[0][1], wz = P[2][2] - P[0][2];
    double nx = uy * wz - uz * wy, ny = uz * wx - ux * wz, nz = ux * wy - uy * wx;
    const double nn = sqrt(nx * nx + ny * ny + nz * nz);
    const double sgn = ((v[f].x - P[0][0]) * nx + (v[f].y - P[0][1]) * ny + (v[f].z - P[0][2]) * nz) < 0 ? -1.0 : 1.0;
    const int i = atomicAdd(count, 1);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) tri[9 * (size_t)i + 3 * a + b] = (float)P[a][b];
    for (int b = 0; b < 3; ++b) pin[3 * (size_t)i + b] = (float)((P[0][b] + P[1][b] + P[2][b]) / 3.0);
    nrm[3 * (size_t)i] = (float)(sgn * nx / nn);
    nrm[3 * (size_t)i + 1] = (float)(sgn * ny / nn);
    nrm[3 * (size_t)i + 2] = (float)(sgn * nz / nn);
    slot[i] = q;
  }
}
__global__ void k_iota(int* p, int n) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) p[k] = k;
}
// shrunk spheres -> the slots' table entries on the 2^-20 grid (centre rounded, radius rounded down so the ball stays
// empty); a sphere that does not fit the site range stays unused
__global__ void k_scatter_spheres(const float4* sph, const int* slot, int n, float4* table, int* used) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const float4 s = sph[k];
    const float x = rintf(s.x * 1048576.0f) * (1.0f / 1048576.0f), y = rintf(s.y * 1048576.0f) * (1.0f / 1048576.0f),
                z = rintf(s.z * 1048576.0f) * (1.0f / 1048576.0f), r = floorf(s.w * 1048576.0f) * (1.0f / 1048576.0f);
    const bool ok = fabsf(x) <= 1.f && fabsf(y) <= 1.f && fabsf(z) <= 1.f && r >= 0.f && r <= 2.f;
    table[slot[k]] = make_float4(x, y, z, r);
    used[slot[k]] = ok ? 0 : 1;
  }
}

hipError_t launch_surface_faces(const float4* tp, const int* tn, int nt, float* tri, float* pin, float* nrm, int* slot,
                                int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_surface_faces, dim3(gsz(4 * (size_t)nt)), dim3(256), 0, s, tp, tn, nt, tri, pin, nrm, slot,
                     count);
  return hipGetLastError();
}
hipError_t launch_iota(int* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(gsz(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
hipError_t launch_scatter_spheres(const float4* sph, const int* slot, int n, float4* table, int* used, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_spheres, dim3(gsz(n)), dim3(256), 0, s, sph, slot, n, table, used);
  return hipGetLastError();
}

// the round's selection and insertion (everything before the clip passes)
hipError_t launch_round_front(const RoundState& r, const ShapeArgs& a, const int* cell_b0,
                              const float4* tp, int nt, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(64), 0, s, r);
  hipLaunchKernelGGL(k_select, dim3(1), dim3(256), 0, s, r, a.cell_chi, a.cell_np, cell_b0);
  const int scan = std::min(r.cnseg, SCAN_BLOCKS);
  hipLaunchKernelGGL(k_ref_tet, dim3(scan), dim3(256), sizeof(unsigned long long) * r.max_insert, s, a.N, r);
  hipLaunchKernelGGL(k_pick_tet, dim3(scan), dim3(256), sizeof(unsigned long long) * r.max_insert, s, a.N, cell_b0,
                     r, tp, a.site);
  hipLaunchKernelGGL(k_insert, dim3(1), dim3(1024), 0, s, r, (float4*)a.site);
  hipLaunchKernelGGL(k_mark_dirty, dim3(gsz(nt)), dim3(256), 0, s, r, tp, nt, a.site, a.tet_U);
  hipLaunchKernelGGL(k_dirty_items, dim3(gsz(nblk)), dim3(256), 0, s, r, nblk);
  return hipGetLastError();
}

hipError_t launch_round_end(const RoundState& r, hipStream_t s) {
  hipLaunchKernelGGL(k_round_end, dim3(1), dim3(64), 0, s, r);
  return hipGetLastError();
}

}  // namespace rpd
