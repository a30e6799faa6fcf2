// Host-side launchers of the librpd kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "rpd_common.h"

namespace rpd {

// clip.hip
hipError_t launch_clip_fast(const ShapeArgs& a, int precision, int block, int slots, hipStream_t s);
size_t slow_scratch_bytes(int waves);
// the item count is read on the device from counters[C_DEFER_ITEMS] (no host synchronisation)
hipError_t launch_clip_slow(const ShapeArgs& a, unsigned char* scratch, int waves, hipStream_t s);

// reduce.hip
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, size_t n, hipStream_t s);
struct FillJob {
  void* p;
  unsigned long long v, v2;  // the value (width 4 or 8), or the two halves of a 16-byte pattern
  size_t n;
  int width;  // 4, 8 or 16 bytes (16: p 16-byte aligned)
};
struct FillList {
  FillJob job[24];
  int n;
  bool overflow;  // more than 24 jobs were added (launch_fill_multi then fails)
  void add(void* ptr, unsigned long long val, size_t count, int w, unsigned long long val2 = 0) {
    if (!count) return;
    if (n < 24) job[n++] = FillJob{ptr, val, val2, count, w};
    else overflow = true;
  }
  // zero counters [c0, c0 + n0) and [c1, c1 + n1) of each of the copies of the statistics (NCOUNTERS apart): a job
  // of width 0 with the four bounds packed in val
  void add_stats_zero(unsigned long long* stats, int copies, int c0, int n0, int c1, int n1) {
    const unsigned long long packed = (unsigned long long)(c0 & 0xffff) | ((unsigned long long)(n0 & 0xffff) << 16) |
                                      ((unsigned long long)(c1 & 0xffff) << 32) |
                                      ((unsigned long long)(n1 & 0xffff) << 48);
    add(stats, packed, (size_t)copies, 0);
  }
};
hipError_t launch_fill_multi(const FillList& L, hipStream_t s);
hipError_t launch_fill_i32(int* p, int v, size_t n, hipStream_t s);
// zero counters [c0, c0 + n0) and [c1, c1 + n1) in every spread copy of the statistics
hipError_t launch_zero_stats(unsigned long long* stats, int c0, int n0, int c1, int n1, hipStream_t s);
// union-find over the live element pieces (with a.touch_* set: only the pieces of touched elements); list [cap N]
// and seg [cap N / 256] receive those pieces' slots per segment of the table (glue_segment_length slots); clist and
// cseg, if not null, the same for every live cell piece
hipError_t launch_glue(const ShapeArgs& a, int* list, int* seg, int* clist, int* cseg, hipStream_t s);
unsigned glue_segment_length(size_t cap);
hipError_t launch_clear_touched_b0(const unsigned char* touch, int* b0, size_t n, hipStream_t s);
// elements of pieces an incremental update removed and did not put back are flagged as touched
hipError_t launch_touch_removed(const ShapeArgs& a, hipStream_t s);
// components per element: the roots among the pieces launch_glue listed
hipError_t launch_count_roots(const ShapeArgs& a, const int* list, const int* seg, int* cell_b0, int* face_b0,
                              int* edge_b0, hipStream_t s);
// the live entries of the face and edge tables (keys and slots) and the counted RPVs (as site quadruples), each
// compacted in any order (its count += their number), in one launch
struct CompactLists {
  struct Live {
    const unsigned long long* keys;
    const int* np;
    unsigned cap, cpt;  // cpt: set by the launcher
    unsigned long long* out_keys;
    int* out_slots;
    unsigned long long* count;
  } live[2];
  HashTab Q;
  const int* rpv_cnt;
  const unsigned long long* ekeys;
  unsigned rpv_cpt;  // set by the launcher
  int4* rpv_out;
  unsigned long long* rpv_count;
  int* zero;     // or null: n_zero ints set to 0 in the same launch (the row sort's counters)
  size_t n_zero;
};
hipError_t launch_compact_lists(CompactLists J, hipStream_t s);
// three lists of keys whose row (key >> shift) is below rows, sorted ascending in place; tmp[l] holds n[l] keys;
// off holds 3 (rows + 1) ints, cur 3 rows ints
// (off and cur must be zero; list 2 is built from the RPV quadruples rpv: keys[2] receives their (j, k, l) keys
// sorted by (i, j, k, l) and rpv_row their first sites i; tsum holds 3 row_tiles(rows) ints of scratch)
int row_tiles(int rows);
hipError_t launch_row_sort(unsigned long long* const keys[3], unsigned long long* const tmp[3],
                           const unsigned long long* n, const size_t ncap[3], const int shift[3], int rows, int* off,
                           int* cur, const int4* rpv, int* rpv_row, int* tsum, hipStream_t s);
// the collect step's four last steps in one launch: face and edge lists over the sorted keys (slots looked up by
// key), the sorted RPVs as quadruples, and the cells
struct FinalizeRows {
  const unsigned long long *fkeys, *ekeys, *qkeys;
  const int* qrows;  // the first site of each sorted RPV
  HashTab F, E;
  const long long *face_chi, *edge_chi, *edge_len, *cell_chi, *cell_geo;
  const int *face_b0, *edge_b0, *cell_np, *cell_b0;
  const float4* site;
  int ns;
};
hipError_t launch_finalize_rows(const FinalizeRows& R, size_t ncap, const OutDesc& od, const ShapeDesc* shapes,
                                int nshapes, int* status, hipStream_t s);
hipError_t launch_validate_sites(const float* sx, const float* sy, const float* sz, const float* sr, int ns,
                                 float4* site, int* status, hipStream_t s);
// the sites of every shape of a call in one launch (src: device array of nsrc records, max_n = the largest n)
struct SiteSrc {
  const float *x, *y, *z, *r;
  int n, off;
};
hipError_t launch_validate_sites_multi(const SiteSrc* src, int nsrc, int max_n, float4* site, int* status,
                                       hipStream_t s);
// the output buffer's face, edge and RPV lists of a batch: per-shape run starts (-1 where a shape has no element)
// and keys turned into each shape's own site ids (ncap: the largest list capacity)
hipError_t launch_localize_lists(const OutDesc& od, size_t ncap, const ShapeDesc* shapes, int nshapes, hipStream_t s);


// session.hip
hipError_t launch_surface_faces(const float4* tp, const int* tn, int nt, float* tri, float* pin, float* nrm, int* slot,
                                int* count, hipStream_t s);
hipError_t launch_iota(int* p, int n, hipStream_t s);
hipError_t launch_scatter_spheres(const float4* sph, const int* slot, int n, float4* table, int* used, hipStream_t s);
void shrink_spheres(const float* tri, long long nt, const float* pins, const float* normals, const int* own,
                    long long n, hipStream_t st, float4* out);
// selection, insertion and dirty marking of one round; a supplies the element tables and sites of the new shape
hipError_t launch_round_front(const RoundState& r, const ShapeArgs& a, const int* cell_b0,
                              const float4* tp, int nt, int nblk, hipStream_t s);
hipError_t launch_round_end(const RoundState& r, hipStream_t s);

}  // namespace rpd
