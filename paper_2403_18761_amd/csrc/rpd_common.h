// Internal structures shared by the host runtime and the kernels of librpd (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpd {

// Fast-path capacities of the clipping kernel.
constexpr int TB = 64;       // tets per workgroup
constexpr int KMAX = 28;     // candidate sites per tet (plane ids 4 + position must fit 5 bits)
constexpr int VMAX = 16;     // vertex slots of one piece (4-bit neighbour ids)
constexpr int SLMAX = 256;   // sites in a workgroup's shared candidate list
// Large-capacity (deferred) path.
constexpr int SLOW_KMAX = 1020;  // candidate sites per tet
constexpr int SLOW_VMAX = 64;    // vertex slots of one piece
constexpr int SLOW_PMAX = 4 + SLOW_KMAX;

// status bits raised by kernels (ShapeArgs::status)
constexpr int ST_DEGENERATE = 1;     // an exact predicate evaluated to zero / duplicate site
constexpr int ST_TABLE_FULL = 2;     // a hash table or record buffer ran out of room (host retries larger)
constexpr int ST_INTERNAL = 4;       // gluing asymmetry or another broken invariant
constexpr int ST_SLOW_CAPACITY = 8;  // the deferred path ran out of candidate or vertex capacity
constexpr int ST_INVALID = 16;       // invalid site value (off grid, out of range, not finite)

// counters (ShapeArgs::counters)
enum { C_PAIRS = 0, C_CAND, C_FP64, C_EXACT, C_DEFER_ITEMS, C_GLUE, C_RPV, C_PIECES, C_NODES, NCOUNTERS };

constexpr unsigned long long EMPTY_KEY = ~0ull;

struct HashTab {
  unsigned long long* keys;  // EMPTY_KEY when free
  unsigned int mask;         // capacity - 1, capacity a power of two
};

// per-piece record kept with RPD_KEEP_PIECES
struct PieceRec {
  int t;  // internal tet id
  int i;  // site
  float vol, mx, my, mz;
  long long chi;  // fractional cell contribution (numerator over L)
};

struct ShapeArgs {
  // ---- mesh, internal (spatially sorted) tet order
  int nt;
  const int* blk;        // [nblk + 1] first tet of every workgroup block (spatially compact runs of <= TB tets)
  int nblk;
  const float4* tp;      // [4 nt] tet vertex coordinates (w unused)
  const int* tn;         // [4 nt] neighbour tet across local face f (face f is opposite vertex f), -1 on the boundary
  const unsigned* nu;    // [14 nt] weight numerators L/k: 4 vertices, 6 edges, 4 faces
  long long L;
  // ---- sites
  int ns;
  const float4* site;    // [ns] (x, y, z, r)
  // ---- accumulators
  long long* cell_chi;   // [ns] fractional chi numerators
  long long* cell_geo;   // [4 ns] volume and first moment, fixed point 2^-56
  int* cell_np;          // [ns] nonempty pieces
  HashTab F;             // faces (i<j): key i<<32 | j
  long long* face_chi;   // [cap F]
  HashTab E;             // edges (i<j<k): key i<<42 | j<<21 | k
  long long* edge_chi;   // [cap E]
  int4* rpv;             // RPV quadruples
  int rpv_cap;
  HashTab N;             // element pieces (union-find nodes): kind<<62 | elem<<32 | tet
  int* node_glue;        // [cap N] bit f set: the element piece touches local face f of its tet (glue across it)
  int2* deferred;        // (tet, site or -1 for every candidate) for the large-capacity path
  int deferred_cap;
  PieceRec* pieces;
  int piece_cap;
  unsigned long long* counters;  // [NCOUNTERS]
  int* status;
  unsigned flags;        // RPD_FORCE_* / RPD_KEEP_PIECES as in rpd.h
  int kmax;              // fast-path candidate budget (<= KMAX)
};

}  // namespace rpd
