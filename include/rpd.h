/*
 * rpd.h -- C ABI of the MI355X restricted-power-diagram library (librpd.so).
 *
 * Computes, for medial spheres (weighted sites) over a tetrahedral mesh of a solid, the volumetric restricted power
 * diagram (RPD) together with the Euler characteristic and the number of connected components of every restricted
 * power cell (RPC), face (RPF) and edge (RPE), and the dual adjacency (which pairs, triples and quadruples of sites
 * meet inside the solid).
 *
 * Definitions followed (paper: MATTopo, Sec. 3.2-3.3, 4.1, 5.2):
 *   - site i = sphere (c_i, r_i), power distance d_i(x) = |x - c_i|^2 - r_i^2 (Sec. 3.2, power-cell equation);
 *   - closed power cell Omega_i = {x : d_i(x) <= d_j(x) for all j != i};
 *   - RPC_i = Omega_i & S with S the union of the input tets; RPF_ij = RPC_i & RPC_j; RPE_ijk = RPF_ij & RPC_k;
 *     RPV_ijkl likewise (Sec. 3.2, duality list);
 *   - chi = V - E + F - C of any cell decomposition (Sec. 4.1, Euler formula), evaluated with the fractional Euler
 *     characteristic of Sec. 4.1.2 (weights 1/k inherited from the mesh simplex carrying each clipped element);
 *   - beta0 = number of connected components (Sec. 4.1.1);
 *   - volume and centroid of each RPC (Lebesgue measure and first moment over S).
 *
 * Input preconditions (Sec. 3.3, Assumption): a manifold tetrahedral mesh with one connected component and no
 * cavity. This library additionally requires:
 *   - every coordinate and radius is a finite float32 on the dyadic grid 2^-20 with |coordinate| <= 1 and
 *     0 <= radius <= 2 (exact integer predicates then have fixed width);
 *   - tets are positively oriented: det(v1-v0, v2-v0, v3-v0) > 0;
 *   - exact ties (a vertex of a clipped piece exactly on a clipping plane: a mesh vertex on a bisector, five
 *     co-spherical sites, equal spheres) are broken by symbolic perturbation of the weights: site s's squared radius
 *     becomes r_s^2 + eps_s with eps_0 >> eps_1 >> ... > 0, so a lower site id wins a tie; the result is the
 *     diagram of that perturbed input (zero-measure pieces included), identical on every code path.
 *
 * Threading: calls on different handles may run concurrently; calls that share a handle must be serialised.
 * All functions return an rpd_status; on a negative status no output is produced (*out is set to NULL) and
 * rpd_last_error() (thread-local) describes the failure.
 */
#ifndef RPD_H
#define RPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rpd_status;

#define RPD_OK 0
#define RPD_E_INVALID (-1)    /* bad argument: NaN/Inf, off-grid value, r < 0, index out of range, bad orientation */
#define RPD_E_MESH (-2)       /* face shared by more than two tets, several components, simplex multiplicity lcm too big */
#define RPD_E_DEGENERATE (-3) /* three clipping planes without a single meet point (cannot occur for valid input) */
#define RPD_E_NOMEM (-4)      /* device or host allocation failed */
#define RPD_E_DEVICE (-5)     /* HIP runtime error or no device */
#define RPD_E_INTERNAL (-6)   /* an internal consistency check failed (gluing asymmetry, non-integer chi, ...) */

/* precision of the clipping constructions */
#define RPD_FP32_FALLBACK 0 /* FP32 clipping; predicates not certified in FP32 are re-done in FP64, then exactly */
#define RPD_FP64 1          /* FP64 clipping; predicates not certified in FP64 are re-done exactly */

/* element kinds */
#define RPD_CELL 1
#define RPD_FACE 2
#define RPD_EDGE 3
#define RPD_VERTEX 4 /* RPV quadruples (adjacency only) */

/* rpd_opts.flags */
#define RPD_DEVICE_PTRS (1u << 0)       /* every input pointer is a device pointer (e.g. a torch tensor's data_ptr) */
#define RPD_FORCE_FP64 (1u << 1)        /* test-only: treat every FP32 predicate as uncertain (go to FP64) */
#define RPD_FORCE_EXACT (1u << 2)       /* test-only: treat every floating-point predicate as uncertain (go exact) */
#define RPD_FORCE_SLOW_PATH (1u << 3)   /* test-only: send every tet through the large-capacity deferred path */
#define RPD_TIMING (1u << 4)            /* record per-kernel HIP-event timings into rpd_stats */
#define RPD_KEEP_PIECES (1u << 5)       /* keep per-piece records (rpd_pieces) for sampled comparisons */
#define RPD_OWNER_WEIGHTS (1u << 6)     /* rpd_mesh_create: ownership weights even when L / k(sigma) fits (below) */
#define RPD_SHUFFLE_QUEUE (1u << 7)     /* test-only: process the work items in a shuffled order (same results) */
#define RPD_ESTIMATED_ORDER (1u << 8)   /* order the work by the static estimate even when a mesh has measured times */
#define RPD_NO_SPLIT (1u << 9)          /* never dispatch a heavy workgroup block in parts (same results, for timing) */

/*
 * A prepared tet mesh (device resident): vertex/tet arrays, face adjacency, the multiplicity k(sigma) of every
 * vertex, edge and face, the fractional weights L/k(sigma) (Sec. 4.1.2) and a spatial ordering of the tets.
 * Created once and reused by every rpd_build on that mesh (the paper recomputes the RPD many times per model).
 * Meshes whose lcm L of multiplicities reaches 2^31 (general, non-voxel tet meshes), or any mesh created with
 * RPD_OWNER_WEIGHTS, use ownership weights instead: a simplex weighs 1 in its owner tet (the lowest caller index
 * among the tets containing it) and 0 in the others, with L = 1. Both sum to weight 1 per simplex over its tets,
 * so every chi is the same; only the per-piece numerators differ.
 */
typedef struct rpd_mesh rpd_mesh;

typedef struct rpd_mesh_desc {
  int32_t n_verts;
  const float *vx, *vy, *vz; /* [n_verts] */
  int32_t n_tets;
  const int32_t* tv;         /* [4 * n_tets], vertex indices, positively oriented */
} rpd_mesh_desc;

typedef struct rpd_mesh_info {
  int32_t n_verts, n_tets, n_edges, n_faces;
  int32_t euler;             /* V - E + F - C of the mesh */
  int32_t components;
  int64_t L;                 /* lcm of all simplex multiplicities: the fixed-point denominator of chi (1 with
                                ownership weights) */
  double volume;
  int32_t owner_weights;     /* 1 if the mesh uses ownership weights */
  int32_t n_blocks;          /* workgroup blocks (spatially compact runs of up to 64 tets) */
} rpd_mesh_info;

typedef struct rpd_sites {
  int32_t n_sites;
  const float *sx, *sy, *sz, *sr; /* [n_sites] centres and radii */
} rpd_sites;

typedef struct rpd_opts {
  int32_t precision;   /* RPD_FP32_FALLBACK or RPD_FP64 */
  int32_t clip_budget; /* max candidate sites per tet in the fast path: 0 = tuned or 28, else 4..28; tets
                          with more go to the large-capacity kernel */
  int32_t block;       /* threads per workgroup of the FP32 clipping kernel: 0 = tuned or 128, 64, 128 or 256
                          (the FP64 path always runs 64) */
  uint32_t flags;      /* RPD_* flags above */
  void* stream;        /* hipStream_t to run on; NULL = the null stream */
  int32_t slots;       /* vertex slots per piece polytope of the 64-thread FP32 clipping kernel: 0 = tuned or 16;
                          16 (six workgroups per compute unit) or 12 (eight: two waves per SIMD, at the cost of
                          more pieces redone with 64 slots and more blocks split); blocks of 128 or 256 threads
                          and the FP64 path use 16. Every value gives the same elements */
} rpd_opts;

typedef struct rpd_stats {
  int64_t n_pairs;        /* nonempty pieces P_{t,i} = tet & Omega_i */
  int64_t n_candidates;   /* (tet, site) pairs clipped in the fast path */
  int64_t n_deferred;     /* (tet, site) items sent to the large-capacity path */
  int64_t n_fp64;         /* predicates re-evaluated in FP64 */
  int64_t n_exact;        /* predicates decided exactly */
  int64_t n_cells, n_faces, n_edges, n_rpv;
  int64_t n_glue;         /* gluing records */
  double ms_clip;         /* HIP-event time of the fast clipping kernel (RPD_TIMING) */
  double ms_deferred;     /* deferred kernel */
  double ms_reduce;       /* gluing, union-find, compaction and sorting */
  double ms_total;        /* whole rpd_build on the stream */
  int64_t n_defer_block;  /* tets deferred because their own candidates overflow the fast path's site list */
  int64_t n_defer_kmax;   /* tets deferred because more candidates than the clip budget remained */
  int64_t n_defer_clip;   /* pieces deferred by the fast path: a predicate undecided in FP64, or over 64 vertices */
  int64_t n_split;        /* workgroup blocks redone in smaller chunks because their site list overflowed */
  int64_t n_items;        /* work items of the fast kernel (blocks, and parts of blocks that were heavy before) */
  int64_t n_big;          /* pieces over the fast path's 16 vertex slots, redone there with a 64-slot polytope */
} rpd_stats;

typedef struct rpd_result rpd_result;

/* Validate and preprocess a mesh (Sec. 4.1.2: weights derived from the combinatorial structure of the tet mesh).
 * Pointers are borrowed (host, or device with RPD_DEVICE_PTRS in flags) and only read during the call.
 * Errors: RPD_E_INVALID (off-grid or out-of-range values, bad indices, non-positive orientation),
 * RPD_E_MESH (a face in more than two tets, more than one component, lcm of multiplicities of 2^31 or more). */
rpd_status rpd_mesh_create(const rpd_mesh_desc* desc, uint32_t flags, void* stream, rpd_mesh** out);
/* A mesh keeps one piece of mutable state: the time each of its blocks took in the last rpd_build that used it,
 * which orders the next build's work (heaviest first). It changes no result. Builds that share a mesh may run
 * from several threads (the hint is locked); rpd_mesh_free must not overlap a build that uses the mesh. */
rpd_status rpd_mesh_get_info(const rpd_mesh* mesh, rpd_mesh_info* info);
void rpd_mesh_free(rpd_mesh* mesh);

/* Compute the RPD, chi and beta0 of n_shapes (mesh, sites) pairs in one call (Sec. 5.2 Tet-Cell clipping, Sec. 4.1).
 * meshes[s] and sites[s] describe shape s (n_shapes in [1, 2^16)); sites pointers are borrowed (host, or device
 * with RPD_DEVICE_PTRS).
 * The result owns every array reachable from it until rpd_free; results are host-visible when the call returns
 * (the stream is synchronised once at the end). Errors: RPD_E_INVALID, RPD_E_DEGENERATE, RPD_E_NOMEM,
 * RPD_E_DEVICE, RPD_E_INTERNAL; no partial result. */
rpd_status rpd_build(const rpd_mesh* const* meshes, const rpd_sites* sites, int32_t n_shapes, const rpd_opts* opts,
                     rpd_result** out);

/* chi of every nonempty element of one kind (RPD_CELL: one entry per site, empty cells report 0).
 * keys: kind site ids per element, ascending within an element; elements sorted lexicographically by key.
 * Returned pointers are host memory owned by the result. (Sec. 4.1.2 / Sec. 4.1 Euler formula.) */
rpd_status rpd_euler(const rpd_result* r, int32_t shape, int32_t kind, int64_t* n_out, const int32_t** keys,
                     const int32_t** chi);

/* beta0 per element, same order as rpd_euler (Sec. 4.1.1). Empty cells report 0. */
rpd_status rpd_components(const rpd_result* r, int32_t shape, int32_t kind, int64_t* n_out, const int32_t** keys,
                          const int32_t** beta0);

/* Volume [n_sites] and centroid [3 * n_sites] of every RPC (empty cell: 0 and NaN). Host memory owned by r. */
rpd_status rpd_geometry(const rpd_result* r, int32_t shape, const double** vol, const double** centroid);

/* Dual adjacency: the element keys of one kind (RPD_FACE pairs, RPD_EDGE triples, RPD_VERTEX quadruples)
 * (Sec. 3.2, RPC/RPF/RPE/RPV duality). */
rpd_status rpd_adjacency(const rpd_result* r, int32_t shape, int32_t kind, int64_t* n_out, const int32_t** keys);

/* Length of every RPE (the summed lengths of its pieces' segments) and the importance of its dual medial triangle,
 * alpha_ijk = |RPE_ijk| / mean diameter 2 r of spheres i, j, k (Sec. 5.3, thinning order). Same order as
 * rpd_euler(RPD_EDGE); alpha is +inf when all three radii are 0. FP32 path: segment lengths from the FP32 piece
 * vertices, summed in 2^-56 fixed point (deterministic). Host memory owned by r. */
rpd_status rpd_edge_geometry(const rpd_result* r, int32_t shape, int64_t* n_out, const double** length,
                             const double** alpha);

/* The dual medial mesh (Sec. 3.2 duality: cell -> vertex, RPF -> edge, RPE -> triangle, RPV -> tet) is given by the
 * key lists above; counts = {V, E, F, T} with V the sites whose cell is nonempty, and chi = V - E + F - T (the
 * medial mesh's Euler characteristic, Sec. 6). counts: room for 4. */
rpd_status rpd_medial_euler(const rpd_result* r, int32_t shape, int64_t* counts, int64_t* chi);

/* Geometry-guided thinning of a simplicial complex (Sec. 5.3), on host arrays (a sequential greedy process; the
 * library runs it on the calling thread). Input: n_vertices, and edges (2 ids), triangles (3 ids) with their
 * importance alpha, tets (4 ids), each simplex's ids strictly ascending and each list sorted lexicographically
 * (the order rpd_adjacency returns); every face of a listed simplex must be listed. Steps:
 *   1. while a tet-face simple pair exists (a triangle with exactly one tet left on it), remove the one with the
 *      least alpha of the triangle (ties: lower triangle index), tet and triangle together;
 *   2. then, among triangles that were faces of the original tets, while a face-edge simple pair (an edge with
 *      exactly one triangle left on it, that triangle on no tet) has alpha < sigma, remove the one with the least
 *      alpha (ties: lower triangle, then lower edge index), triangle and edge together.
 * Vertices are never removed; every removal keeps the Euler characteristic. Output: keep masks (1 = kept) of
 * n_edges, n_tris and n_tets bytes, caller-owned; tets that no simple pair could reach stay kept.
 * Errors: RPD_E_INVALID (unsorted or out-of-range ids, a missing face, NaN alpha or sigma, null arrays),
 * RPD_E_NOMEM. */
rpd_status rpd_thin(int32_t n_vertices, int64_t n_edges, const int32_t* edges, int64_t n_tris, const int32_t* tris,
                    const double* alpha, int64_t n_tets, const int32_t* tets, double sigma, uint8_t* keep_edge,
                    uint8_t* keep_tri, uint8_t* keep_tet);

/* Distance from surface samples to the enveloping volume of a medial mesh (Sec. 4.3, geometric preservation; the
 * enveloping elements of Sec. 3.2: a vertex's sphere, an edge's medial cone, a triangle's medial slab, i.e. the
 * spheres interpolated linearly over the simplex). For sample q and element e with spheres B(c(t), r(t)):
 * value_e(q) = min over t of |q - c(t)| - r(t), the distance to e's volume when q is outside it (negative inside);
 * dist[s] = min over all elements, nearest[s] = the element reaching it (ties: lowest id), ids numbered spheres
 * 0..n_spheres-1, then edges, then triangles. No element: dist = +inf, nearest = -1.
 * spheres: 4 floats per sphere (x, y, z, r); edges: 2 sphere ids each; tris: 3 sphere ids each; every face of a
 * listed edge or triangle must be listed too (an element is evaluated at its interior stationary point and leaves
 * its boundary to those faces, which is exact for a closed complex such as the output of rpd_thin).
 * samples: 3 floats per sample. With RPD_DEVICE_PTRS in flags every array (inputs and outputs) is device memory
 * and the call runs on stream (NULL = the null stream); otherwise host memory. nearest may be NULL. FP32
 * arithmetic (element constants rounded from FP64). kernel_ms (host, may be NULL): HIP-event time of the distance
 * kernel on that stream. Synchronises the stream.
 * Errors: RPD_E_INVALID (negative count, null array, sphere id out of range), RPD_E_NOMEM, RPD_E_DEVICE. */
rpd_status rpd_envelope_distance(const float* spheres, int32_t n_spheres, const int32_t* edges, int64_t n_edges,
                                 const int32_t* tris, int64_t n_tris, const float* samples, int64_t n_samples,
                                 uint32_t flags, void* stream, float* dist, int32_t* nearest, float* kernel_ms);

/* No-allocation variant of rpd_envelope_distance, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation). Same arguments and results as
 * rpd_envelope_distance with RPD_DEVICE_PTRS (every array is device memory, the call runs on stream, NULL = the null
 * stream, nearest may be NULL), without kernel timing; it runs the same kernels and gives the same bits. Its working
 * memory (element records, per-sample minima, a status word) lives in a fixed region of RPD_NOALLOC_SCRATCH_BYTES
 * on each device, reserved with the library's code and held until the process ends; the call itself allocates
 * nothing. Limit: 256 + 8 n_samples + 16 (3 n_edges + 5 n_tris) bytes, each part rounded up to 256, must fit the
 * region (else RPD_E_NOMEM, checked before any device work). All calls on one device share the region and every call
 * rewrites what it uses: calls that overlap on one device (from other host threads or on other streams) race, so
 * the caller serialises them. Synchronises the stream (to read the status word).
 * Errors: RPD_E_INVALID (negative count, null array, sphere id out of range), RPD_E_NOMEM (over the limit),
 * RPD_E_DEVICE. */
#define RPD_NOALLOC_SCRATCH_BYTES (64u << 20)
rpd_status rpd_envelope_distance_noalloc(const float* spheres, int32_t n_spheres, const int32_t* edges,
                                         int64_t n_edges, const int32_t* tris, int64_t n_tris, const float* samples,
                                         int64_t n_samples, void* stream, float* dist, int32_t* nearest);

/* Medial spheres by sphere shrinking (Sec. 5.1, Fig. tech_sphere_gen (a)): for each pin point p with inward unit
 * normal n, the maximal ball tangent to the surface at p with no surface point inside, i.e. the fixed point of the
 * shrinking iteration. The surface is given as triangles (9 floats each: three vertices); the radius is
 * min over surface points q with n.(q - p) > 0 of |q - p|^2 / (2 n.(q - p)), computed exactly per triangle
 * (vertices, edge stationary points, plane tangency) over all triangles. own_tri (may be NULL): per pin, the index
 * of the triangle that carries it (excluded). Output: 4 floats per pin (centre p + r n, radius r; r = +inf when no
 * surface point lies on the inner side). FP32 arithmetic, constants rounded from FP64. With RPD_DEVICE_PTRS every
 * array is device memory and the call runs on stream; otherwise host memory. Synchronises the stream.
 * Errors: RPD_E_INVALID (negative count, null array), RPD_E_NOMEM, RPD_E_DEVICE. */
rpd_status rpd_shrink_spheres(const float* tris, int64_t n_tris, const float* pins, const float* normals,
                              const int32_t* own_tri, int64_t n_pins, uint32_t flags, void* stream, float* spheres);

/* Counters of the call (summed over shapes). */
rpd_status rpd_get_stats(const rpd_result* r, rpd_stats* stats);

/* Per-piece records kept with RPD_KEEP_PIECES: for every nonempty piece (tet t in the caller's numbering, site i):
 * vol, first moment (3), and the fractional chi numerator of its cell contribution (over L). n_out pieces;
 * arrays are host memory owned by r, ordered by (t, i). */
rpd_status rpd_pieces(const rpd_result* r, int32_t shape, int64_t* n_out, const int32_t** tet, const int32_t** site,
                      const double** vol_moment /* 4 per piece */, const int64_t** chi_num);

/* Per-piece element terms kept with RPD_KEEP_PIECES (Sec. 4.1.2: each piece's fractional contributions; Sec. 4.1.1:
 * the mesh faces through which its element pieces are glued). kind RPD_CELL: one term per nonempty piece (site i;
 * num = its cell contribution over L; glue bit f: the piece touches interior face f of its tet, bit 4 + f: boundary
 * face f). RPD_FACE: one per face of a piece lying on the bisector of i against j > i (sites i, j; num = the RPF
 * piece's contribution; glue bit f: the face polygon has an edge on interior face f). RPD_EDGE: one per segment of
 * a piece on the bisectors of i against j and k, i < j < k (sites i, j, k; glue bit f: an endpoint on interior face
 * f). RPD_VERTEX: one per vertex of a piece on three bisectors, all of whose sites exceed i (sites i, j, k, l; num 1,
 * glue 0). tet is in the caller's numbering; sites holds kind ids per term (shape-local); terms are ordered by
 * (tet, sites). Arrays are host memory owned by r; n_out is 0 without RPD_KEEP_PIECES. */
rpd_status rpd_piece_terms(const rpd_result* r, int32_t shape, int32_t kind, int64_t* n_out, const int32_t** tet,
                           const int32_t** sites, const int64_t** num, const int32_t** glue);

void rpd_free(rpd_result* r);

/* Autotuner for the batched FP32 path: runs rpd_build on these inputs once per launch shape (block of 64, 128 or 256
 * threads x clip budget 8, 16 or 28 with 16 vertex slots, and 64 threads with 12 slots x budget 16 or 28), each
 * timed by HIP events over the clipping kernels, best of two after a warm-up, writes the fastest into *best (a copy
 * of *opts with block, clip_budget and slots set; the default 64 x 28 x 16 is kept unless another shape is more than
 * 2% faster) and caches it for the process under the bucket (floor log2 of the mean sites per shape, floor log2 of
 * the mean tets per shape). Later rpd_build calls take the cached value of their bucket for each of block,
 * clip_budget and slots that is 0 (else 64, 28 and 16), and so does a session. Every launch shape gives the same
 * elements (keys, chi, beta0); a piece that one shape defers to the large-capacity kernel and another does not has
 * its geometry built in FP64 instead of FP32, which can move volumes and moments in their last bits. Synchronises.
 * Errors as rpd_build; RPD_E_INVALID for RPD_FP64. */
rpd_status rpd_autotune(const rpd_mesh* const* meshes, const rpd_sites* sites, int32_t n_shapes, const rpd_opts* opts,
                        rpd_opts* best);

/* ---- Incremental session: the sphere-insertion loop of topology repair (Sec. 4 overview: spheres are added where
 * an element violates the topology constraints, and only the cells related to the new spheres are updated).
 *
 * A session keeps the RPD of one mesh and a growing site set resident on the device. Every round
 *   1. selects up to max_insert restricted power cells with chi != 1 or more than one component (lowest site ids
 *      first; Sec. 3.3 / 4.1 criteria for a cell),
 *   2. picks for each a tet among the cell's pieces (for a cell with several components, outside the component
 *      of its piece in the smallest tet, tets in the caller's numbering) and appends a sphere (each at most once):
 *      RPD_INSERT_TABLE: the sphere that `table` holds for the candidate tet t (pieces whose table sphere is not in
 *      yet) with the largest pair (h, t), h = the upper 32 bits of the splitmix64 finaliser of t * 2^32 + round
 *      (rounds counted from 0); spheres are appended in the order of the selected cells, a cell's sphere skipped
 *      when an earlier cell of the round picked the same tet;
 *      RPD_INSERT_SHRINK (Sec. 4.1.3 with Sec. 5.1): among the surface triangles (mesh faces without a neighbour)
 *      the cell's pieces touch, the one whose centroid is furthest from the cell's sphere centre is the pin, and the
 *      sphere is the shrunk sphere at that pin (rpd_shrink_spheres over the mesh surface, computed once at
 *      creation and rounded to the 2^-20 grid: centre to nearest, radius down);
 *   3. re-clips only the workgroup blocks whose tets a new sphere can reach (exact candidate test), removing the
 *      blocks' old contributions and adding the new ones, and recomputes the components.
 * The round is one captured HIP graph replayed by rpd_session_run. The state after any number of rounds is
 * identical, bit for bit, to rpd_build on the same mesh with the session's current sites (rpd_session_sites).
 */
typedef struct rpd_session rpd_session;

#define RPD_INSERT_TABLE 0  /* insertion from the caller's per-tet table */
#define RPD_INSERT_SHRINK 1 /* insertion by sphere shrinking at the furthest surface triangle of the cell */

typedef struct rpd_session_opts {
  int32_t max_sites;  /* capacity: initial sites plus every insertion, in [n_sites, 2^21) */
  int32_t max_insert; /* cells handled per round, 1..4096 */
  rpd_opts build;     /* precision, clip_budget, block, flags as for rpd_build (RPD_DEVICE_PTRS applies to the sites
                         and the table); build.stream is synchronised before the session reads the inputs, and the
                         session then runs on a stream of its own */
  int32_t insertion;  /* RPD_INSERT_TABLE or RPD_INSERT_SHRINK */
} rpd_session_opts;

typedef struct rpd_session_info {
  int32_t n_sites;        /* sites in use */
  int32_t rounds;         /* rounds run so far */
  int32_t n_selected;     /* cells selected in the last round */
  int32_t n_blocks;       /* workgroup blocks of the mesh */
  int64_t n_inserted;     /* spheres inserted over all rounds */
  int64_t n_dirty_blocks; /* blocks re-clipped over all rounds */
  int64_t n_clipped;      /* (tet, candidate site) pairs clipped since creation, removal passes included */
  double ms_last_run;     /* HIP-event time of the last rpd_session_run */
} rpd_session_info;

/* Create a session: validate the inputs, compute the initial RPD, capture the round graph.
 * mesh is borrowed and must outlive the session. sites: the initial spheres. table (RPD_INSERT_TABLE; NULL with
 * RPD_INSERT_SHRINK): one sphere per tet of the mesh in the caller's tet order (table->n_sites == n_tets), on the
 * 2^-20 grid like every site. Synchronises.
 * Errors: RPD_E_INVALID, RPD_E_DEGENERATE, RPD_E_NOMEM, RPD_E_DEVICE. */
rpd_status rpd_session_create(const rpd_mesh* mesh, const rpd_sites* sites, const rpd_sites* table,
                              const rpd_session_opts* opts, rpd_session** out);

/* Run `rounds` rounds (graph replays), then synchronise and check the device status (ties with an inserted sphere
 * are broken like every other tie, see the preconditions above). Errors: RPD_E_NOMEM (the session's tables filled
 * up: create it with a larger max_sites), RPD_E_DEVICE. After an error the session can only be freed. */
rpd_status rpd_session_run(rpd_session* s, int32_t rounds);

/* The current state as an rpd_result (shape 0), read with the accessors above and released with rpd_free. */
rpd_status rpd_session_result(rpd_session* s, rpd_result** out);

rpd_status rpd_session_get_info(rpd_session* s, rpd_session_info* info);

/* Copy the current sites (x, y, z, r per site, in site-id order) into host memory xyzr of room for cap sites. */
rpd_status rpd_session_sites(rpd_session* s, int32_t cap, float* xyzr, int32_t* n_out);

void rpd_session_free(rpd_session* s);

/* Thread-local description of the last error of this thread ("" if none). */
const char* rpd_last_error(void);

/* Library version string. */
const char* rpd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RPD_H */
