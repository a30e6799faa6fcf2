// Internal structures shared by the host runtime and the kernels of librpd (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpd {

// Fast-path capacities of the clipping kernel.
constexpr int TB = 64;       // tets per workgroup
constexpr int KMAX = 28;     // candidate sites per tet kept for clipping (plane ids 4 + position must fit 5 bits)
constexpr int KRAW = 40;     // candidate sites per tet before the dominance refinement
constexpr int VMAX = 16;     // vertex slots of one piece (4-bit neighbour ids)
constexpr int SLMAX = 256;   // sites in a workgroup's shared candidate list
constexpr int SUB = 8;       // tets per chunk when a block's site list overflows
// Work items are (shape + (tet mask << 16), block + (part << ITEM_PART_SHIFT)): part 0 is the whole block, part
// p >= 1 its tets [(p - 1) SPLIT_TETS, p SPLIT_TETS) (heavy blocks are dispatched in parts so that no workgroup sets
// the kernel's tail). A nonzero tet mask (parts only) names the part's tets to clip, bit k for its tet k; zero
// means all. Shapes per call < 2^16.
constexpr int ITEM_PART_SHIFT = 20;  // blocks per mesh < 2^20
constexpr int SPLIT_TETS = 16;       // = the width of the tet mask
// Large-capacity (deferred) path.
constexpr int SLOW_KMAX = 1020;  // candidate sites per tet
constexpr int SLOW_VMAX = 64;    // vertex slots of one piece
constexpr int SLOW_PMAX = 4 + SLOW_KMAX;
// Fast-path pieces that outgrow VMAX vertex slots are redone in the same kernel with a global-memory polytope of
// BIG_VCAP slots (coordinates + bound in the kernel's precision, 64-bit topology words, a byte per plane for the
// pairing table).
constexpr int BIG_VCAP = 64;
constexpr size_t BIG_BYTES = 32 * BIG_VCAP + 8 * BIG_VCAP + 64;

// status bits raised by kernels (ShapeArgs::status)
constexpr int ST_DEGENERATE = 1;     // an exact predicate evaluated to zero / duplicate site
constexpr int ST_TABLE_FULL = 2;     // a hash table or record buffer ran out of room (host retries larger)
constexpr int ST_INTERNAL = 4;       // gluing asymmetry or another broken invariant
constexpr int ST_SLOW_CAPACITY = 8;  // the deferred path ran out of candidate or vertex capacity
constexpr int ST_INVALID = 16;       // invalid site value (off grid, out of range, not finite)

// counters (ShapeArgs::counters)
enum {
  C_PAIRS = 0, C_CAND, C_FP64, C_EXACT, C_DEFER_ITEMS, C_GLUE, C_RPV, C_PIECES, C_NODES,
  C_DEFER_BLOCK,  // tets deferred because their own candidates overflow the workgroup's site list
  C_DEFER_KMAX,   // tets deferred because they kept more than the candidate budget
  C_DEFER_CLIP,   // pieces deferred because the polytope outgrew the vertex slots
  C_SPLIT,        // workgroup blocks redone in chunks because their site list overflowed
  C_DEFER2,       // items handed on by the LDS variant of the large-capacity kernel
  C_GLUE_BITS,    // gluing bits of the pieces whose components are (re)computed
  C_GLUE_PAIRS,   // glued pairs matched
  C_TERMS,        // per-piece element terms kept with RPD_KEEP_PIECES (cursor)
  C_LISTS,        // candidate lists handed from the fast kernel to the large-capacity kernel (cursor)
  C_BIG,          // pieces the fast kernel redid in a global-memory polytope after running out of slots (cursor;
                  // follows C_LISTS: an incremental pass resets both together)
  NCOUNTERS
};
// C_RPV counts RPV emissions; the RPV list itself is the set of keys of ShapeArgs::Q with a positive count

// Statistics counters are spread over NSPREAD copies (picked by workgroup id) so that thousands of workgroups do
// not serialise on one address; the host sums the copies. Counters used as cursors (C_DEFER_ITEMS, C_PIECES) are
// not spread.
constexpr int NSPREAD = 64;

constexpr unsigned long long EMPTY_KEY = ~0ull;

// element-piece state word
// element-piece state: NODE_UNIT x (times the piece was emitted) + 16 x (boundary faces of the tet the piece touches,
// cells only) + gluing bits (interior faces of the tet the piece touches)
constexpr int NODE_UNIT = 256;
__host__ __device__ inline bool node_live(int st) { return st >= NODE_UNIT; }
__host__ __device__ inline int node_glue_bits(int st) { return st & 15; }
__host__ __device__ inline int node_bnd_bits(int st) { return (st >> 4) & 15; }

struct HashTab {
  unsigned long long* keys;  // EMPTY_KEY when free
  unsigned int mask;         // capacity - 1, capacity a power of two
};

// Element pieces (the union-find nodes), one 16-byte record per slot: an insert, its state update and the gluing
// pass's lookups of a piece touch one cache line.
struct NodeRec {
  unsigned long long key;  // kind << 62 | element << 32 | batch-global tet, EMPTY_KEY when free
  int st;                  // NODE_UNIT x (times the piece is present) + boundary bits + gluing bits
  int parent;              // union-find parent slot
};
struct NodeTab {
  NodeRec* rec;
  unsigned int mask;  // capacity - 1, capacity a power of two
};

// The byte layout of the one buffer that carries a call's results to the host, a function of the site count, the
// shape count and the live face, edge and RPV counts (so that kernels can place their output from the counts in
// device memory before the host knows them): doubles first, then the RPVs (int4), then the int32 arrays.
struct OutLayout {
  size_t vol, cen, elen, ealpha, rpv, cchi, cb0, fk, fchi, fb0, ek, echi, eb0, start, bytes;
};
__host__ __device__ inline OutLayout out_layout(size_t ns, size_t nsh, size_t nf, size_t ne, size_t nq) {
  OutLayout L;
  size_t o = 0;
  L.vol = o;
  o += 8 * ns;
  L.cen = o;
  o += 24 * ns;
  L.elen = o;
  o += 8 * ne;
  L.ealpha = o;
  o += 8 * ne;
  o = (o + 15) / 16 * 16;
  L.rpv = o;
  o += 16 * nq;
  L.cchi = o;
  o += 4 * ns;
  L.cb0 = o;
  o += 4 * ns;
  L.fk = o;
  o += 8 * nf;
  L.fchi = o;
  o += 4 * nf;
  L.fb0 = o;
  o += 4 * nf;
  L.ek = o;
  o += 12 * ne;
  L.echi = o;
  o += 4 * ne;
  L.eb0 = o;
  o += 4 * ne;
  L.start = o;  // [3][nsh] first face, edge and RPV of every shape (batches)
  o += 12 * nsh;
  L.bytes = (o + 15) / 16 * 16;
  return L;
}
// The output buffer as kernels see it: base, site and shape counts, and the live counts [faces, edges, RPVs] in
// device memory.
struct OutDesc {
  unsigned char* base;
  const unsigned long long* n;
  int ns, nsh;
  __device__ OutLayout layout() const { return out_layout(ns, nsh, n[0], n[1], n[2]); }
};

// per-piece record kept with RPD_KEEP_PIECES
struct PieceRec {
  int t;  // internal tet id
  int i;  // site
  float vol, mx, my, mz;
  long long chi;  // fractional cell contribution (numerator over L)
};

// per-piece element term kept with RPD_KEEP_PIECES: the piece of site i in tet t contributes num (over L) to the
// element of kind 1 (cell i), 2 (face {i, j}), 3 (edge {i, j, k}) or 4 (RPV {i, j, k, l}: num = 1), and touches the
// faces of t in glue (bit f: interior face f; cells also 16 << f: boundary face f)
struct TermRec {
  int kind, t, i, j, k, l, glue, pad;
  long long num;
};

// One shape of a batch: its prepared mesh and its range of the batch's site array.
struct ShapeDesc {
  const float4* tp;    // [4 nt] tet vertex coordinates (w unused), internal (Morton) tet order
  const double4* tf;   // [4 nt] face f of every tet in FP64, tet-local frame (normal exact, offset rounded once)
  const int* tn;       // [4 nt] neighbour tet across local face f (face f is opposite vertex f), -1 on the boundary
  const unsigned* nu;  // [14 nt] weight numerators L/k: 4 vertices, 6 edges, 4 faces
  const int* blk;      // [nblk + 1] first tet of every workgroup block (spatially compact runs of <= TB tets)
  int nt, nblk;
  long long L;
  int site_off, ns;    // sites [site_off, site_off + ns) of the batch
  long long tet_off;   // batch-global id of the shape's tet 0
  int sign;            // +1: the shape's pieces are added; -1: an incremental update takes them back (the state
                       // before the round's insertions)
  int pad;
};

// Everything the kernels of one rpd_build call share. Site ids and tet ids in keys and accumulators are
// batch-global (a shape's local id plus its offset), so one set of tables serves every shape.
struct ShapeArgs {
  const ShapeDesc* shapes;
  int nshapes;
  const int2* items;     // (shape, block and part) work items, heaviest first
  int nitems;            // number of items, or the grid size when nitems_dev is set
  const int* nitems_dev; // optional: the item count in device memory (graph-captured rounds)
  // ---- sites (all shapes)
  int ns;
  const float4* site;    // [ns] (x, y, z, r)
  // ---- accumulators
  long long* cell_chi;   // [ns] fractional chi numerators
  long long* cell_geo;   // [8 ns] volume and first moment: 128-bit fixed point 2^-80 as (low, high) word pairs
  int* cell_np;          // [ns] nonempty pieces
  HashTab F;             // faces (i<j, global ids): key i<<32 | j
  long long* face_chi;   // [cap F]
  int* face_np;          // [cap F] pieces (the face exists while > 0)
  HashTab E;             // edges (i<j<k, global ids < 2^21): key i<<42 | j<<21 | k
  long long* edge_chi;   // [cap E]
  int* edge_np;          // [cap E]
  long long* edge_len;   // [cap E] summed RPE piece lengths, 2^-56 units
  HashTab Q;             // RPVs (i<j<k<l): key edge slot of (i,j,k) << 21 | l
  int* rpv_cnt;          // [cap Q] (exists while > 0)
  NodeTab N;             // element pieces (union-find nodes); a piece is emitted once per pass, so adding its
                         // gluing bits (bit f: glue across local face f of its tet) to the state equals or-ing them
  // optional (incremental update): element flags set by every emission, so that only the components of touched
  // elements are recomputed; indexed by site (cells), face-table slot and edge-table slot
  unsigned char* touch_cell;
  unsigned char* touch_face;
  unsigned char* touch_edge;
  unsigned short* removed;  // [2 cap N] with touch flags: per element-piece slot, 0x100 | the gluing bits with which
                            // an incremental update took the piece out (even entry) and put it back (odd entry)
  double* tet_U;         // optional [total tets]: U_t of the candidate test, kept for the incremental update
  int4* deferred;        // (shape, local tet, global site or -1 for every candidate, list) for the large-capacity
                         // path; list = 64 x (index in deferred_list) + m when the fast kernel hands over the tet's
                         // m sorted candidates, else 0 (the large-capacity kernel then finds them itself)
  int deferred_cap;
  int* deferred_list;    // [list_cap][KRAW] batch-global site ids
  int list_cap;
  unsigned char* big;    // [big_cap][BIG_BYTES] global-memory polytopes of the fast kernel's overflowing pieces
  int big_cap;
  int4* deferred2;       // items the LDS variant of the large-capacity path hands to its global variant
  int deferred2_cap;
  PieceRec* pieces;      // kept with RPD_KEEP_PIECES (t = global tet id)
  int piece_cap;
  TermRec* terms;        // kept with RPD_KEEP_PIECES (t = global tet id)
  int term_cap;
  unsigned long long* counters;  // [NCOUNTERS] (cursors and host-read totals)
  unsigned long long* stats;     // [NSPREAD][NCOUNTERS] spread statistics
  int* status;
  unsigned flags;        // RPD_FORCE_* / RPD_KEEP_PIECES as in rpd.h
  int kmax;              // fast-path candidate budget (<= KMAX)
  unsigned* item_cost;   // optional [nitems]: wall-clock ticks each work item took in the fast kernel
};

// shape of a batch-global id by binary search over the shapes' offsets
__device__ inline int shape_of_site(const ShapeDesc* sd, int n, int gi) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sd[mid].site_off <= gi) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
__device__ inline int shape_of_tet(const ShapeDesc* sd, int n, long long gt) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sd[mid].tet_off <= gt) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}


// Device state of one round of the incremental session (all counts live in device memory so that the round is a
// fixed launch sequence).
constexpr int MAX_INSERT = 4096;  // cells handled per session round, at most

struct RoundState {
  int* nsel;                  // cells selected this round
  int* sel;                   // [max_insert] selected cells, ascending
  int* selpos;                // [max_sites] position of a cell in sel, or -1
  unsigned long long* best;   // [max_insert] packed (hash, slot) of the slot chosen for the cell
  unsigned long long* ref;    // [max_insert] the cell's piece in its smallest tet: caller tet << 32 | internal tet
  int* tet_used;              // [slots] the slot's sphere has been inserted (or it has none)
  const float4* table;        // [slots] the sphere of every slot: per tet in the caller's numbering (mode 0) or per
                              // (internal tet, face) (mode 1)
  const int* perm;            // [nt] internal -> caller tet
  int mode;                   // 0: caller's per-tet table, hashed pick; 1: shrunk spheres at the furthest surface face
  const int* tet_block;       // [nt] workgroup block of every tet
  unsigned long long* dirty;  // [nblk] per block, the mask of its dirty tets (bit k: the block's tet k)
  const int* order;           // [nblk] blocks by their time in the initial build, heaviest first (scan order)
  const int* blk;             // [nblk + 1] first tet of every block
  int2* items;                // [8 nblk] dirty (shape 0 or 1 and tet mask, block part) items, in about that order
  const int* clist;           // the live cell pieces' slots, per segment of clen table slots (the gluing pass
  const int* cseg;            // writes them): cseg[b] of them at clist[b clen]
  unsigned clen;
  int cnseg;
  int* nitems;
  int* round;
  int* ns_cur;                // sites in use
  int* ins_total;             // spheres inserted over all rounds
  int* dirty_total;           // dirty blocks over all rounds
  ShapeDesc* old_desc;        // the shape with the sites before this round's insertions
  ShapeDesc* new_desc;        // ... and after them
  int max_sites;
  int max_insert;
};

__device__ inline void stat_add(const ShapeArgs& a, int c, unsigned long long v) {
  atomicAdd(&a.stats[(blockIdx.x & (NSPREAD - 1)) * NCOUNTERS + c], v);
}
__device__ inline unsigned long long stat_sum(const ShapeArgs& a, int c) {
  unsigned long long v = 0;
  for (int k = 0; k < NSPREAD; ++k) v += a.stats[k * NCOUNTERS + c];
  return v;
}

}  // namespace rpd
