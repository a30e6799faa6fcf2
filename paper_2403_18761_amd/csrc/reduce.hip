// Reductions after clipping: connected components by union-find over glued element pieces (paper Sec. 4.1.1),
// integer Euler characteristics from the fractional sums (Sec. 4.1.2), compaction and sorting of the element lists,
// site validation and small fills.
#include <algorithm>
#include <cstring>

#include <hip/hip_runtime.h>

#include "rpd_device.h"
#include "rpd_launch.h"

namespace rpd {

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = v;
}
__global__ void k_fill_i32(int* p, int v, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = v;
}

// several fills in one launch (blockIdx.y = job): each job writes n values of 4 or 8 bytes (p aligned to the
// width), with 16-byte stores between the first and the last 16-byte boundary and single values around them
__global__ void k_fill_multi(FillList L) {
  const FillJob j = L.job[blockIdx.y];
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x, step = (size_t)gridDim.x * blockDim.x;
  if (j.width == 0) {  // counters of every copy of the statistics (FillList::add_stats_zero)
    const int c0 = (int)(j.v & 0xffff), n0 = (int)((j.v >> 16) & 0xffff), c1 = (int)((j.v >> 32) & 0xffff),
              n1 = (int)(j.v >> 48);
    unsigned long long* st = (unsigned long long*)j.p;
    for (size_t k = tid; k < j.n; k += step) {
      for (int c = 0; c < n0; ++c) st[k * NCOUNTERS + c0 + c] = 0;
      for (int c = 0; c < n1; ++c) st[k * NCOUNTERS + c1 + c] = 0;
    }
    return;
  }
  if (j.width == 16) {  // a 16-byte pattern over a 16-byte aligned array
    const uint4 val = make_uint4((unsigned)j.v, (unsigned)(j.v >> 32), (unsigned)j.v2, (unsigned)(j.v2 >> 32));
    for (size_t k = tid; k < j.n; k += step) ((uint4*)j.p)[k] = val;
    return;
  }
  const unsigned lo = (unsigned)j.v, hi = j.width == 8 ? (unsigned)(j.v >> 32) : lo;
  const size_t w = (size_t)j.width;
  const size_t head = min(((16 - ((size_t)j.p & 15)) & 15) / w, j.n);  // values before the first boundary
  const size_t nvec = (j.n - head) * w / 16;
  const size_t tail0 = head + nvec * 16 / w;  // first value after the last full 16 bytes
  if (tid < head || (tid >= head && tid - head < j.n - tail0)) {
    const size_t k = tid < head ? tid : tail0 + (tid - head);
    if (w == 8) ((unsigned long long*)j.p)[k] = j.v;
    else ((unsigned*)j.p)[k] = lo;
  }
  uint4* q = (uint4*)((unsigned char*)j.p + head * w);
  const uint4 val = make_uint4(lo, hi, lo, hi);
  for (size_t k = tid; k < nvec; k += step) q[k] = val;
}

static int grid_for(size_t n, int bs) {
  size_t g = (n + bs - 1) / bs;
  if (g > 65536) g = 65536;
  return (int)(g ? g : 1);
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
// counters [c0, c0 + n0) and [c1, c1 + n1) in every spread copy of the statistics
__global__ void k_zero_stats(unsigned long long* stats, int c0, int n0, int c1, int n1) {
  const int k = threadIdx.x;  // one thread per spread copy
  if (k < NSPREAD) {
    for (int c = 0; c < n0; ++c) stats[(size_t)k * NCOUNTERS + c0 + c] = 0;
    for (int c = 0; c < n1; ++c) stats[(size_t)k * NCOUNTERS + c1 + c] = 0;
  }
}
hipError_t launch_zero_stats(unsigned long long* stats, int c0, int n0, int c1, int n1, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(NSPREAD), 0, s, stats, c0, n0, c1, n1);
  return hipGetLastError();
}

hipError_t launch_fill_multi(const FillList& L, hipStream_t s) {
  if (L.overflow) return hipErrorInvalidValue;
  if (L.n <= 0) return hipSuccess;
  size_t big = 1;  // 16-byte vectors of the largest job (at least one thread per value outside them)
  for (int k = 0; k < L.n; ++k) big = std::max(big, std::max(L.job[k].n * L.job[k].width / 16, (size_t)8));
  hipLaunchKernelGGL(k_fill_multi, dim3(std::min(grid_for(big, 256), 1024), L.n), dim3(256), 0, s, L);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* p, int v, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------------------------
// union-find (lock-free: hook the larger root under the smaller with CAS; path halving)
// ---------------------------------------------------------------------------------------------------------------
__device__ inline int uf_find(NodeRec* rec, int x) {
  while (true) {
    int p = rec[x].parent;
    if (p == x) return x;
    int gp = rec[p].parent;
    if (gp != p) rec[x].parent = gp;
    x = p;
  }
}
__device__ inline void uf_union(NodeRec* rec, int a, int b) {
  while (true) {
    a = uf_find(rec, a);
    b = uf_find(rec, b);
    if (a == b) return;
    if (a < b) {
      int t = a;
      a = b;
      b = t;
    }
    int old = atomicCAS(&rec[a].parent, a, b);
    if (old == a) return;
  }
}

// with touch flags (incremental update) only the pieces of touched elements are redone: unions never join two
// elements, so the forest of every other element stays valid
__device__ inline bool node_touched(const ShapeArgs& a, unsigned long long key) {
  if (!a.touch_cell) return true;
  const int kind = node_kind(key), elem = node_elem(key);
  return (kind == 1 ? a.touch_cell : kind == 2 ? a.touch_face : a.touch_edge)[elem] != 0;
}

// Output position of a thread's n items: exclusive prefix within the 256-thread block, plus the block's base from
// one global atomic per block (a wave-level atomic on one address for every wave of a large table serialises).
__device__ inline unsigned long long block_append(int n, unsigned long long* count) {
  __shared__ int s_w[4];
  __shared__ unsigned long long s_base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = n;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_w[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    s_base = tot ? atomicAdd(count, (unsigned long long)tot) : 0ull;
  }
  __syncthreads();
  int before = 0;
  for (int q = 0; q < w; ++q) before += s_w[q];
  return s_base + (unsigned long long)(before + x - n);
}

// One scan of the element-piece table: every live piece whose element is redone becomes its own root and goes on
// the gluing list (gluing and root counting then visit the list, not the table); live pieces are counted and every
// state word is checked (each piece present at most once). Workgroup b (256 threads) scans the slots of segment b,
// [b len, (b + 1) len), and lists its pieces in the same range of the list, seg[b] of them: no global cursor, and
// the later passes give segment b to workgroup b. The segment length grows with the table (at least 256 slots, at
// most 4,096 segments), which bounds the workgroups' statistics atomics.
__global__ __launch_bounds__(256) void k_parent_init(ShapeArgs a, int* list, int* seg, int* clist, int* cseg,
                                                     unsigned len) {
  __shared__ unsigned long long s_n, s_nc;
  if (threadIdx.x == 0) s_n = s_nc = 0;
  __syncthreads();
  unsigned long long nodes = 0;
  const unsigned base = blockIdx.x * len;  // the table holds a whole number of segments
  for (unsigned run = 0; run < len; run += 256) {
    const unsigned s = base + run + threadIdx.x;
    const NodeRec r = a.N.rec[s];
    const int st = r.key == EMPTY_KEY ? 0 : r.st;
    if (st < 0 || st >= 2 * NODE_UNIT) atomicOr(a.status, ST_INTERNAL);
    const bool live = node_live(st);
    nodes += live ? 1 : 0;
    const bool take = live && node_touched(a, r.key);
    if (take) a.N.rec[s].parent = (int)s;
    const unsigned long long pos = block_append(take ? 1 : 0, &s_n);
    if (take) list[base + pos] = (int)s;
    __syncthreads();  // block_append's shared words are rewritten by the next call
    if (clist) {  // every live cell piece, for the next incremental round's selection scans
      const bool cell = live && node_kind(r.key) == 1;
      const unsigned long long cpos = block_append(cell ? 1 : 0, &s_nc);
      if (cell) clist[base + cpos] = (int)s;
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    seg[blockIdx.x] = (int)s_n;
    if (cseg) cseg[blockIdx.x] = (int)s_nc;
  }
  __shared__ unsigned long long s_nodes;
  if (threadIdx.x == 0) s_nodes = 0;
  __syncthreads();
  if (nodes) atomicAdd(&s_nodes, nodes);
  __syncthreads();
  if (threadIdx.x == 0 && s_nodes) stat_add(a, C_NODES, s_nodes);
}

// pieces an incremental update took out and did not put back with the same gluing bits, or added new: their
// elements are flagged
__global__ void k_touch_removed(ShapeArgs a) {
  const unsigned cap = a.N.mask + 1;
  unsigned* pair = (unsigned*)a.removed;  // (taken out, put back) tags of a slot in one word
  for (unsigned s = blockIdx.x * blockDim.x + threadIdx.x; s < cap; s += gridDim.x * blockDim.x) {
    const unsigned w = pair[s];
    if (!w) continue;
    pair[s] = 0;
    if ((w & 0xffffu) == (w >> 16)) continue;
    const unsigned long long key = a.N.rec[s].key;
    const int kind = node_kind(key), elem = node_elem(key);
    (kind == 1 ? a.touch_cell : kind == 2 ? a.touch_face : a.touch_edge)[elem] = 1;
  }
}
hipError_t launch_touch_removed(const ShapeArgs& a, hipStream_t s) {
  const size_t cap = (size_t)a.N.mask + 1;
  hipLaunchKernelGGL(k_touch_removed, dim3(grid_for(cap, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ void k_clear_touched_b0(const unsigned char* touch, int* b0, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    if (touch[k]) b0[k] = 0;
}

// For every element piece with gluing bits: find the same element's piece in the face-adjacent tet, check that it
// glues back across the same mesh face (both sides must agree), and unite them.
// Every gluing bit is matched from the tet with the smaller id only (one lookup and one union per glued pair); the
// symmetry of the records is checked by counting: the bits set must be twice the pairs matched.
__global__ void k_glue(ShapeArgs a, const int* list, const int* seg, unsigned len) {
  // the shapes' first tets, for the lookup of a piece's shape in LDS (up to 256 shapes; more search in memory)
  constexpr int LS = 256;
  __shared__ long long s_toff[LS];
  const bool local = a.nshapes > 1 && a.nshapes <= LS;
  if (local)
    for (int k = threadIdx.x; k < a.nshapes; k += blockDim.x) s_toff[k] = a.shapes[k].tet_off;
  __syncthreads();
  const int n = seg[blockIdx.x];
  unsigned long long bits = 0, pairs = 0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int s = list[(size_t)blockIdx.x * len + k];
    const NodeRec r = a.N.rec[s];
    const unsigned long long key = r.key;
    int g = node_glue_bits(r.st);
    if (!g) continue;
    bits += __popc(g);
    const long long gt = (long long)(key & 0xffffffffull);
    int sh = 0;
    if (local) {  // the last shape whose first tet is at most gt
      int lo = 0, hi = a.nshapes - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_toff[mid] <= gt) lo = mid;
        else hi = mid - 1;
      }
      sh = lo;
    } else if (a.nshapes > 1) {
      sh = shape_of_tet(a.shapes, a.nshapes, gt);
    }
    const ShapeDesc& sd = a.shapes[sh];
    const int t = (int)(gt - sd.tet_off);
    unsigned long long hi = key & ~0xffffffffull;
    const int4 nb = reinterpret_cast<const int4*>(sd.tn)[t];  // the four face neighbours, one 16-byte load
    for (int f = 0; f < 4; ++f) {
      if (!(g & (1 << f))) continue;
      const int t2 = f == 0 ? nb.x : f == 1 ? nb.y : f == 2 ? nb.z : nb.w;
      if (t2 < t) continue;  // the boundary never carries a bit; the other side matches smaller ids
      const int4 nb2 = reinterpret_cast<const int4*>(sd.tn)[t2];
      const int f2 = nb2.x == t ? 0 : nb2.y == t ? 1 : nb2.z == t ? 2 : nb2.w == t ? 3 : -1;
      int s2 = node_find(a.N, hi | (unsigned)(sd.tet_off + t2));
      const int st2 = s2 >= 0 ? a.N.rec[s2].st : 0;
      if (s2 < 0 || f2 < 0 || !node_live(st2) || !(node_glue_bits(st2) & (1 << f2))) {
        atomicOr(a.status, ST_INTERNAL);
        continue;
      }
      ++pairs;
      uf_union(a.N.rec, s, s2);
    }
  }
  __shared__ unsigned long long s_sum[2];
  if (threadIdx.x < 2) s_sum[threadIdx.x] = 0;
  __syncthreads();
  if (bits) atomicAdd(&s_sum[0], bits);
  if (pairs) atomicAdd(&s_sum[1], pairs);
  __syncthreads();
  if (threadIdx.x == 0 && s_sum[0]) stat_add(a, C_GLUE_BITS, s_sum[0]);
  if (threadIdx.x == 0 && s_sum[1]) stat_add(a, C_GLUE_PAIRS, s_sum[1]);
}

__global__ void k_count_roots(ShapeArgs a, const int* list, const int* seg, unsigned len, int* cell_b0,
                              int* face_b0, int* edge_b0) {
  const int n = seg[blockIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0 && stat_sum(a, C_GLUE_BITS) != 2 * stat_sum(a, C_GLUE_PAIRS))
    atomicOr(a.status, ST_INTERNAL);  // a gluing bit without its counterpart
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int s = list[(size_t)blockIdx.x * len + k];
    const NodeRec r = a.N.rec[s];
    if (r.parent != s) continue;  // one root per component
    const unsigned long long key = r.key;
    const int kind = (int)(key >> 62);
    const int elem = (int)((key >> 32) & 0x3fffffffull);
    if (kind == 1) atomicAdd(&cell_b0[elem], 1);
    else if (kind == 2) atomicAdd(&face_b0[elem], 1);
    else atomicAdd(&edge_b0[elem], 1);
  }
}

hipError_t launch_clear_touched_b0(const unsigned char* touch, int* b0, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_clear_touched_b0, dim3(grid_for(n, 256)), dim3(256), 0, s, touch, b0, n);
  return hipGetLastError();
}


// segment length of the gluing list: a power of two, at least 256 slots and at most 4,096 segments
static unsigned glue_seg_len(size_t cap) { return (unsigned)std::max<size_t>(256, cap / 4096); }

unsigned glue_segment_length(size_t cap) { return glue_seg_len(cap); }

hipError_t launch_glue(const ShapeArgs& a, int* list, int* seg, int* clist, int* cseg, hipStream_t s) {
  const size_t cap = (size_t)a.N.mask + 1;
  const unsigned len = glue_seg_len(cap);
  hipLaunchKernelGGL(k_parent_init, dim3(cap / len), dim3(256), 0, s, a, list, seg, clist, cseg, len);
  hipLaunchKernelGGL(k_glue, dim3(cap / len), dim3(256), 0, s, a, (const int*)list, (const int*)seg, len);
  return hipGetLastError();
}

hipError_t launch_count_roots(const ShapeArgs& a, const int* list, const int* seg, int* cell_b0, int* face_b0,
                              int* edge_b0, hipStream_t s) {
  const size_t cap = (size_t)a.N.mask + 1;
  const unsigned len = glue_seg_len(cap);
  hipLaunchKernelGGL(k_count_roots, dim3(cap / len), dim3(256), 0, s, a, list, seg, len, cell_b0, face_b0, edge_b0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------------------------
// element lists: compact the live entries of a table (any order), sort exactly those by key, then turn the
// fractional sums into integers
// ---------------------------------------------------------------------------------------------------------------
// Each workgroup takes cpt runs of 256 consecutive slots (lane-strided, so every load is coalesced); cpt grows with
// the table from 1 (small tables: enough workgroups to cover the latency) to 16 (one global atomic per 4,096 slots).
static unsigned compact_cpt(size_t cap) {
  size_t c = (cap + 256 * 2048 - 1) / (256 * 2048);
  return (unsigned)std::min<size_t>(std::max<size_t>(c, 1), 16);
}

__device__ __forceinline__ void compact_live_block(unsigned bx, const unsigned long long* keys, const int* np,
                                                   unsigned cap, unsigned cpt, unsigned long long* out_keys,
                                                   int* out_slots, unsigned long long* count) {
  const size_t q0 = (size_t)bx * cpt * 256 + threadIdx.x;
  int n = 0;
  for (unsigned k = 0; k < cpt; ++k) {
    const size_t q = q0 + 256 * (size_t)k;
    if (q < cap && keys[q] != EMPTY_KEY && np[q] > 0) ++n;
  }
  unsigned long long pos = block_append(n, count);
  for (unsigned k = 0; k < cpt && n; ++k) {
    const size_t q = q0 + 256 * (size_t)k;
    if (q < cap && keys[q] != EMPTY_KEY && np[q] > 0) {
      out_keys[pos] = keys[q];
      out_slots[pos] = (int)q;
      ++pos;
      --n;
    }
  }
}

// RPV quadruples (i, j, k, l) of the counted set (key = edge slot of (i, j, k) << 21 | l), compacted
__device__ __forceinline__ void rpv_compact_block(unsigned bx, const HashTab& Q, const int* cnt,
                                                  const unsigned long long* ekeys, unsigned cpt, int4* out,
                                                  unsigned long long* count) {
  const size_t cap = (size_t)Q.mask + 1;
  const size_t q0 = (size_t)bx * cpt * 256 + threadIdx.x;
  int n = 0;
  for (unsigned k = 0; k < cpt; ++k) {
    const size_t q = q0 + 256 * (size_t)k;
    if (q < cap && Q.keys[q] != EMPTY_KEY && cnt[q] > 0) ++n;
  }
  unsigned long long pos = block_append(n, count);
  for (unsigned k = 0; k < cpt && n; ++k) {
    const size_t q = q0 + 256 * (size_t)k;
    if (q < cap && Q.keys[q] != EMPTY_KEY && cnt[q] > 0) {
      const unsigned long long key = Q.keys[q];
      const unsigned long long e = ekeys[key >> 21];
      out[pos] = make_int4((int)(e >> 42), (int)((e >> 21) & 0x1fffff), (int)(e & 0x1fffff), (int)(key & 0x1fffff));
      ++pos;
      --n;
    }
  }
}

// The three compactions of the collect step in one launch (blockIdx.y: live faces, live edges, counted RPVs); each
// takes the workgroups of x that its table needs, the others return at once.
__global__ __launch_bounds__(256) void k_compact_lists(CompactLists J) {
  const unsigned bx = blockIdx.x;
  if (blockIdx.y == 3) {
    for (size_t k = bx * (size_t)blockDim.x + threadIdx.x; k < J.n_zero; k += (size_t)gridDim.x * blockDim.x)
      J.zero[k] = 0;
    return;
  }
  if (blockIdx.y < 2) {
    const CompactLists::Live& L = J.live[blockIdx.y];
    if ((size_t)bx * L.cpt * 256 >= L.cap) return;
    compact_live_block(bx, L.keys, L.np, L.cap, L.cpt, L.out_keys, L.out_slots, L.count);
  } else {
    if ((size_t)bx * J.rpv_cpt * 256 >= (size_t)J.Q.mask + 1) return;
    rpv_compact_block(bx, J.Q, J.rpv_cnt, J.ekeys, J.rpv_cpt, J.rpv_out, J.rpv_count);
  }
}
hipError_t launch_compact_lists(CompactLists J, hipStream_t s) {
  size_t gx = 1;
  for (int y = 0; y < 2; ++y) {
    J.live[y].cpt = compact_cpt(J.live[y].cap);
    const size_t per = 256 * (size_t)J.live[y].cpt;
    gx = std::max(gx, (J.live[y].cap + per - 1) / per);
  }
  const size_t capQ = (size_t)J.Q.mask + 1;
  J.rpv_cpt = compact_cpt(capQ);
  gx = std::max(gx, (capQ + 256 * (size_t)J.rpv_cpt - 1) / (256 * (size_t)J.rpv_cpt));
  hipLaunchKernelGGL(k_compact_lists, dim3((unsigned)gx, J.zero && J.n_zero ? 4 : 3), dim3(256), 0, s, J);
  return hipGetLastError();
}

// The element lists are sorted by rows, one row per first site: count the keys of every row, scan the counts,
// scatter the keys to their rows, then place each key by its rank within its (short) row. Three lists per launch
// (blockIdx.y selects the list); the row arrays hold 3 x (rows + 1) counts and 3 x rows cursors. Faces and edges
// carry their first site in the key's top bits; an RPV (i, j, k, l) is keyed by (j, k, l) in 63 bits with its row i
// kept beside it (the scatter writes it next to the key's row position, which the ranking only permutes).
struct RowLists {
  unsigned long long* keys[3];  // in: keys (lists 0 and 1; list 2 is built from rpv); out: sorted
  unsigned long long* tmp[3];   // scratch of the same size
  const unsigned long long* n;  // [3] key counts, in device memory
  int shift[3];                 // row = key >> shift (lists 0 and 1)
  int* off;                     // [3][rows + 1]
  int* cur;                     // [3][rows]
  int rows;
  const int4* rpv;              // list 2's RPV quadruples, in any order
  int* rpv_row;                 // [n[2]]: the row (first site) of each sorted position of list 2
  int* tsum;                    // [3][ntiles]: per tile of ROW_TILE counts, the sum of the tiles before it
  int ntiles;
};
constexpr int ROW_TILE = 4096;  // row counts scanned per workgroup
// the first position of row r of list l (the tile's scan plus the tiles before it)
__device__ __forceinline__ int row_start(const RowLists& L, int l, int r) {
  const int v = L.off[l * (L.rows + 1) + r];
  return L.ntiles > 1 ? v + L.tsum[l * L.ntiles + r / ROW_TILE] : v;
}
__device__ __forceinline__ unsigned long long rpv_key(const int4& r) {  // (j, k, l), 21 bits each
  return ((unsigned long long)r.y << 42) | ((unsigned long long)r.z << 21) | (unsigned long long)r.w;
}
__global__ void k_row_count(RowLists L) {
  const int l = blockIdx.y, n = (int)L.n[l];
  int* off = L.off + l * (L.rows + 1);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    int row;
    if (l == 2) {
      const int4 r = L.rpv[q];
      L.keys[2][q] = rpv_key(r);
      row = r.x;
    } else {
      row = (int)(L.keys[l][q] >> L.shift[l]);
    }
    atomicAdd(&off[row + 1], 1);
  }
}
// the row counts scanned in place, one tile of ROW_TILE per workgroup (grid.y = list): off[q] held the count of row
// q - 1 and becomes the sum of the counts of the rows before q within its tile; the tile's total goes to tsum
__global__ __launch_bounds__(1024) void k_row_scan(RowLists L) {
  __shared__ int s_v[ROW_TILE];
  __shared__ int s_part[1024];
  const int l = blockIdx.y, t = threadIdx.x;
  int* off = L.off + l * (L.rows + 1);
  const int n = L.rows + 1, base = blockIdx.x * ROW_TILE;
  for (int k = 0; k < ROW_TILE / 1024; ++k) {
    const int q = base + k * 1024 + t;
    s_v[k * 1024 + t] = q < n ? off[q] : 0;
  }
  __syncthreads();
  int v[ROW_TILE / 1024], sum = 0;
  for (int k = 0; k < ROW_TILE / 1024; ++k) {
    sum += s_v[t * (ROW_TILE / 1024) + k];
    v[k] = sum;
  }
  s_part[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan of the per-thread sums
    const int x = t >= d ? s_part[t - d] : 0;
    __syncthreads();
    s_part[t] += x;
    __syncthreads();
  }
  const int run = t ? s_part[t - 1] : 0;
  for (int k = 0; k < ROW_TILE / 1024; ++k) s_v[t * (ROW_TILE / 1024) + k] = run + v[k];
  __syncthreads();
  for (int k = 0; k < ROW_TILE / 1024; ++k) {
    const int q = base + k * 1024 + t;
    if (q < n) off[q] = s_v[k * 1024 + t];
  }
  if (t == 1023 && L.ntiles > 1) L.tsum[l * L.ntiles + blockIdx.x] = s_part[1023];
}
// the tile totals of each list turned into the sums of the tiles before each (one workgroup per list)
__global__ __launch_bounds__(1024) void k_row_tiles(RowLists L) {
  __shared__ int s_part[1024];
  const int l = blockIdx.x, t = threadIdx.x;
  int* ts = L.tsum + l * L.ntiles;
  const int x0 = t < L.ntiles ? ts[t] : 0;
  s_part[t] = x0;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int x = t >= d ? s_part[t - d] : 0;
    __syncthreads();
    s_part[t] += x;
    __syncthreads();
  }
  if (t < L.ntiles) ts[t] = s_part[t] - x0;
}
__global__ void k_row_scatter(RowLists L) {
  const int l = blockIdx.y, n = (int)L.n[l];
  int* cur = L.cur + l * L.rows;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const unsigned long long k = L.keys[l][q];
    const int r = l == 2 ? L.rpv[q].x : (int)(k >> L.shift[l]);
    const int pos = row_start(L, l, r) + atomicAdd(&cur[r], 1);
    L.tmp[l][pos] = k;
    if (l == 2) L.rpv_row[pos] = r;
  }
}
// every key finds its place within its row by counting the smaller keys of the row (rows are short; keys unique)
__global__ void k_row_rank(RowLists L) {
  const int l = blockIdx.y, n = (int)L.n[l];
  const unsigned long long* t = L.tmp[l];
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const unsigned long long k = t[q];
    const int r = l == 2 ? L.rpv_row[q] : (int)(k >> L.shift[l]);
    const int a = row_start(L, l, r), b = row_start(L, l, r + 1);
    int rank = 0;
    for (int x = a; x < b; ++x) rank += t[x] < k ? 1 : 0;
    L.keys[l][a + rank] = k;
  }
}
int row_tiles(int rows) { return (rows + 1 + ROW_TILE - 1) / ROW_TILE; }

hipError_t launch_row_sort(unsigned long long* const keys[3], unsigned long long* const tmp[3],
                           const unsigned long long* n, const size_t ncap[3], const int shift[3], int rows, int* off,
                           int* cur, const int4* rpv, int* rpv_row, int* tsum, hipStream_t s) {
  RowLists L;
  size_t nmax = 1;
  for (int l = 0; l < 3; ++l) {
    L.keys[l] = keys[l];
    L.tmp[l] = tmp[l];
    L.shift[l] = shift[l];
    nmax = std::max(nmax, ncap[l]);
  }
  L.n = n;
  const int grid = std::min(grid_for(nmax, 256), 2048);
  L.off = off;
  L.cur = cur;
  L.rows = rows;
  L.rpv = rpv;
  L.rpv_row = rpv_row;
  L.tsum = tsum;
  L.ntiles = row_tiles(rows);
  if (L.ntiles > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_row_count, dim3(grid, 3), dim3(256), 0, s, L);
  hipLaunchKernelGGL(k_row_scan, dim3(L.ntiles, 3), dim3(1024), 0, s, L);
  if (L.ntiles > 1) hipLaunchKernelGGL(k_row_tiles, dim3(3), dim3(1024), 0, s, L);
  hipLaunchKernelGGL(k_row_scatter, dim3(grid, 3), dim3(256), 0, s, L);
  hipLaunchKernelGGL(k_row_rank, dim3(grid, 3), dim3(256), 0, s, L);
  return hipGetLastError();
}

// sorted RPV keys and their rows (see k_row_count) back to quadruples
__device__ __forceinline__ void unpack_rpv_body(int t0, int stride, const unsigned long long* in, const int* row,
                                                const OutDesc& od) {
  const int n = (int)od.n[2];
  int4* out = (int4*)(od.base + od.layout().rpv);
  for (int q = t0; q < n; q += stride) {
    const unsigned long long k = in[q];
    out[q] = make_int4(row[q], (int)(k >> 42), (int)((k >> 21) & 0x1fffff), (int)(k & 0x1fffff));
  }
}

__device__ __forceinline__ void finalize_faces_body(int t0, int stride, const unsigned long long* keys,
                                                    const int* slots, const HashTab& T, const OutDesc& od,
                                                    const long long* chi_num, const int* b0, const ShapeDesc* shapes,
                                                    int nshapes, int* status) {
  const int n = (int)od.n[0];
  const OutLayout L = od.layout();
  int* out_keys = (int*)(od.base + L.fk);
  int* out_chi = (int*)(od.base + L.fchi);
  int* out_b0 = (int*)(od.base + L.fb0);
  for (int q = t0; q < n; q += stride) {
    unsigned long long k = keys[q];
    int s = slots ? slots[q] : ht_find(T, k);
    out_keys[2 * q] = (int)(k >> 32);
    out_keys[2 * q + 1] = (int)(k & 0xffffffffull);
    const long long L = shapes[shape_of_site(shapes, nshapes, (int)(k >> 32))].L;
    long long c = chi_num[s];
    if (c % L != 0) atomicOr(status, ST_INTERNAL);
    out_chi[q] = (int)(c / L);
    out_b0[q] = b0[s];
  }
}
// RPE length (fixed point -> double) and the thinning importance alpha = length / mean diameter of the three spheres
__device__ __forceinline__ void finalize_edges_body(int t0, int stride, const unsigned long long* keys,
                                                    const int* slots, const HashTab& T, const OutDesc& od,
                                                    const long long* chi_num, const int* b0, const long long* len_num,
                                                    const float4* site, const ShapeDesc* shapes, int nshapes,
                                                    int* status) {
  const int n = (int)od.n[1];
  const OutLayout L = od.layout();
  int* out_keys = (int*)(od.base + L.ek);
  int* out_chi = (int*)(od.base + L.echi);
  int* out_b0 = (int*)(od.base + L.eb0);
  double* out_len = (double*)(od.base + L.elen);
  double* out_alpha = (double*)(od.base + L.ealpha);
  for (int q = t0; q < n; q += stride) {
    unsigned long long k = keys[q];
    int s = slots ? slots[q] : ht_find(T, k);
    out_keys[3 * q] = (int)(k >> 42);
    out_keys[3 * q + 1] = (int)((k >> 21) & 0x1fffff);
    out_keys[3 * q + 2] = (int)(k & 0x1fffff);
    const long long L = shapes[shape_of_site(shapes, nshapes, (int)(k >> 42))].L;
    long long c = chi_num[s];
    if (c % L != 0) atomicOr(status, ST_INTERNAL);
    out_chi[q] = (int)(c / L);
    out_b0[q] = b0[s];
    const double len = (double)len_num[s] * (1.0 / 72057594037927936.0);  // 2^-56
    const double dsum = 2.0 * ((double)site[out_keys[3 * q]].w + (double)site[out_keys[3 * q + 1]].w +
                               (double)site[out_keys[3 * q + 2]].w);
    out_len[q] = len;
    out_alpha[q] = dsum > 0.0 ? 3.0 * len / dsum : INFINITY;
  }
}
__device__ __forceinline__ void finalize_cells_body(int t0, int stride, int ns, const long long* chi_num,
                                                    const long long* geo, const int* np, const int* b0,
                                                    const ShapeDesc* shapes, int nshapes, const OutDesc& od,
                                                    int* status) {
  const OutLayout L = od.layout();
  int* out_chi = (int*)(od.base + L.cchi);
  int* out_b0 = (int*)(od.base + L.cb0);
  double* out_vol = (double*)(od.base + L.vol);
  double* out_cen = (double*)(od.base + L.cen);
  for (int i = t0; i < ns; i += stride) {
    const long long L = shapes[shape_of_site(shapes, nshapes, i)].L;
    long long c = chi_num[i];
    if (c % L != 0) atomicOr(status, ST_INTERNAL);
    out_chi[i] = (int)(c / L);
    out_b0[i] = b0[i];
    // 128-bit accumulators (low word, high word) in units of 2^-80
    auto value = [&](int d) {
      const unsigned long long lo = (unsigned long long)geo[8 * (size_t)i + 2 * d];
      const long long hi = geo[8 * (size_t)i + 2 * d + 1];
      return ldexp(ldexp((double)hi, 64) + (double)lo, -80);
    };
    const double v = value(0);
    out_vol[i] = v;
    for (int d = 0; d < 3; ++d) out_cen[3 * (size_t)i + d] = np[i] ? value(1 + d) / v : NAN;
  }
}
// blockIdx.y: faces, edges, RPVs, cells
__global__ void k_finalize_rows(FinalizeRows R, OutDesc od, const ShapeDesc* shapes, int nshapes, int* status) {
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  switch (blockIdx.y) {
    case 0:
      finalize_faces_body(t0, stride, R.fkeys, nullptr, R.F, od, R.face_chi, R.face_b0, shapes, nshapes, status);
      break;
    case 1:
      finalize_edges_body(t0, stride, R.ekeys, nullptr, R.E, od, R.edge_chi, R.edge_b0, R.edge_len, R.site, shapes,
                          nshapes, status);
      break;
    case 2:
      unpack_rpv_body(t0, stride, R.qkeys, R.qrows, od);
      break;
    default:
      finalize_cells_body(t0, stride, R.ns, R.cell_chi, R.cell_geo, R.cell_np, R.cell_b0, shapes, nshapes, od, status);
  }
}
hipError_t launch_finalize_rows(const FinalizeRows& R, size_t ncap, const OutDesc& od, const ShapeDesc* shapes,
                                int nshapes, int* status, hipStream_t s) {
  const int gx = std::min(grid_for(std::max(ncap, (size_t)R.ns), 256), 2048);
  hipLaunchKernelGGL(k_finalize_rows, dim3(gx, 4), dim3(256), 0, s, R, od, shapes, nshapes, status);
  return hipGetLastError();
}



// ---------------------------------------------------------------------------------------------------------------
// site validation: finite, on the 2^-20 grid, |centre| <= 1, 0 <= r <= 2; packs (x, y, z, r)
// ---------------------------------------------------------------------------------------------------------------
__device__ inline bool on_grid(float v, float lim) {
  if (!(fabsf(v) <= lim)) return false;
  float s = v * 1048576.0f;
  return s == rintf(s);
}
__global__ void k_validate_sites(const float* sx, const float* sy, const float* sz, const float* sr, int ns,
                                 float4* site, int* status) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
    float x = sx[i], y = sy[i], z = sz[i], r = sr[i];
    if (!on_grid(x, 1.0f) || !on_grid(y, 1.0f) || !on_grid(z, 1.0f) || !on_grid(r, 2.0f) || r < 0.0f)
      atomicOr(status, ST_INVALID);
    site[i] = make_float4(x, y, z, r);
  }
}
hipError_t launch_validate_sites(const float* sx, const float* sy, const float* sz, const float* sr, int ns,
                                 float4* site, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_validate_sites, dim3(grid_for(ns, 256)), dim3(256), 0, s, sx, sy, sz, sr, ns, site, status);
  return hipGetLastError();
}
// every shape of a call in one launch: shape blockIdx.y
__global__ void k_validate_sites_multi(const SiteSrc* src, float4* site, int* status) {
  const SiteSrc d = src[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.n; i += gridDim.x * blockDim.x) {
    float x = d.x[i], y = d.y[i], z = d.z[i], r = d.r[i];
    if (!on_grid(x, 1.0f) || !on_grid(y, 1.0f) || !on_grid(z, 1.0f) || !on_grid(r, 2.0f) || r < 0.0f)
      atomicOr(status, ST_INVALID);
    site[(size_t)d.off + i] = make_float4(x, y, z, r);
  }
}
hipError_t launch_validate_sites_multi(const SiteSrc* src, int nsrc, int max_n, float4* site, int* status,
                                       hipStream_t s) {
  if (nsrc <= 0 || max_n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate_sites_multi, dim3(std::min(grid_for(max_n, 256), 1024), nsrc), dim3(256), 0, s, src,
                     site, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------------------------
// per-shape runs of the sorted element lists of a batch (elements sorted by batch-global keys: one contiguous run
// per shape), then the keys turned into each shape's own site ids. List y of the launch: faces (2 ids per element),
// edges (3), RPVs (4); start[y][shape] is the first element of the shape, or stays -1 when it has none.
// ---------------------------------------------------------------------------------------------------------------
// the three lists of the output buffer: faces (2 ids per element), edges (3), RPVs (4)
__device__ inline void list_of(const OutDesc& od, const OutLayout& L, int y, int** keys, int* n, int* w) {
  *keys = (int*)(od.base + (y == 0 ? L.fk : y == 1 ? L.ek : L.rpv));
  *n = (int)od.n[y];
  *w = y + 2;
}
__global__ void k_list_starts(OutDesc od, const ShapeDesc* shapes, int nshapes) {
  const OutLayout L = od.layout();
  int* keys;
  int n, w;
  list_of(od, L, blockIdx.y, &keys, &n, &w);
  int* start = (int*)(od.base + L.start) + (size_t)blockIdx.y * nshapes;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const int sh = shape_of_site(shapes, nshapes, keys[(size_t)w * q]);
    if (q == 0 || shape_of_site(shapes, nshapes, keys[(size_t)w * (q - 1)]) != sh) start[sh] = q;
  }
}
__global__ void k_localize(OutDesc od, const ShapeDesc* shapes, int nshapes) {
  const OutLayout L = od.layout();
  int* keys;
  int n, w;
  list_of(od, L, blockIdx.y, &keys, &n, &w);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const int off = shapes[shape_of_site(shapes, nshapes, keys[(size_t)w * q])].site_off;
    for (int c = 0; c < w; ++c) keys[(size_t)w * q + c] -= off;
  }
}
__global__ void k_fill_starts(OutDesc od, int nshapes) {
  int* start = (int*)(od.base + od.layout().start);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < 3 * nshapes; q += gridDim.x * blockDim.x) start[q] = -1;
}
hipError_t launch_localize_lists(const OutDesc& od, size_t ncap, const ShapeDesc* shapes, int nshapes, hipStream_t s) {
  const dim3 grid(std::min(grid_for(ncap, 256), 2048), 3);
  hipLaunchKernelGGL(k_fill_starts, dim3(grid_for(3 * (size_t)nshapes, 256)), dim3(256), 0, s, od, nshapes);
  hipLaunchKernelGGL(k_list_starts, grid, dim3(256), 0, s, od, shapes, nshapes);
  hipLaunchKernelGGL(k_localize, grid, dim3(256), 0, s, od, shapes, nshapes);
  return hipGetLastError();
}

}  // namespace rpd
