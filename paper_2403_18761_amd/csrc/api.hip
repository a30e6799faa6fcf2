// C ABI of librpd (declared in include/rpd.h): argument checking, buffer management, kernel sequencing on the
// caller's stream, and the host copies of the results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "rpd.h"
#include "rpd_host.h"
#include "rpd_launch.h"

namespace rpd {

static thread_local std::string g_error;
void set_error(const std::string& msg) { g_error = msg; }

// ---- caching allocator
static std::mutex g_pool_mu;
static std::map<std::pair<int, size_t>, std::vector<void*>> g_pool;

void* pool_alloc(size_t bytes, size_t* cls_bytes) {
  size_t c = 256;
  while (c < bytes) c <<= 1;
  int dev = 0;
  (void)hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> g(g_pool_mu);
    auto& v = g_pool[{dev, c}];
    if (!v.empty()) {
      void* p = v.back();
      v.pop_back();
      *cls_bytes = c;
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, c);
  if (e == hipErrorOutOfMemory) {  // give cached blocks back to the runtime and try once more
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> g(g_pool_mu);
      for (auto& kv : g_pool)
        for (void* q : kv.second) (void)hipFree(q);
      g_pool.clear();
    }
    e = hipMalloc(&p, c);
  }
  hip_check(e, "hipMalloc");
  *cls_bytes = c;
  return p;
}

void pool_free(void* p, size_t cls_bytes) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(g_pool_mu);
  g_pool[{dev, cls_bytes}].push_back(p);
}

static unsigned pow2_cap(size_t n) {
  size_t c = 1024;
  while (c < n) c <<= 1;
  if (c > (1u << 31)) throw Failure{RPD_E_NOMEM, "table capacity above 2^31"};
  return (unsigned)c;
}

// process-wide scratch of the large-capacity kernel (one region per thread of its grid), grown on demand
static std::mutex g_scratch_mu;
static DBuf g_scratch;
static int g_scratch_device = -1;
constexpr int SLOW_THREADS = 4096;

static unsigned char* slow_scratch() {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  int dev = 0;
  (void)hipGetDevice(&dev);
  size_t need = slow_scratch_bytes(SLOW_THREADS);
  if (g_scratch.p == nullptr || g_scratch.bytes < need || g_scratch_device != dev) {
    g_scratch.alloc(need);
    g_scratch_device = dev;
  }
  return g_scratch.as<unsigned char>();
}

struct ShapeOut {
  int ns = 0;
  std::vector<int32_t> cell_keys, cell_chi, cell_b0;
  std::vector<double> vol, cen;
  std::vector<int32_t> face_keys, face_chi, face_b0;
  std::vector<int32_t> edge_keys, edge_chi, edge_b0;
  std::vector<int32_t> rpv_keys;
  std::vector<int32_t> pc_t, pc_i;
  std::vector<double> pc_geo;
  std::vector<int64_t> pc_chi;
};

struct Timing {
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  bool on = false;
  explicit Timing(bool enable) : on(enable) {
    if (!on) return;
    for (auto& e : ev) hip_check(hipEventCreate(&e), "hipEventCreate");
  }
  ~Timing() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void mark(int k, hipStream_t s) {
    if (on) hip_check(hipEventRecord(ev[k], s), "hipEventRecord");
  }
  double ms(int a, int b) {
    if (!on) return 0.0;
    float x = 0;
    hip_check(hipEventElapsedTime(&x, ev[a], ev[b]), "hipEventElapsedTime");
    return x;
  }
};

template <class T>
static void d2h(std::vector<T>& v, const void* src, size_t n, hipStream_t s) {
  v.resize(n);
  if (n) hip_check(hipMemcpyAsync(v.data(), src, sizeof(T) * n, hipMemcpyDeviceToHost, s), "download");
}

// One shape, one attempt. Returns false if a table ran out of room (caller retries with a larger scale).
static bool run_shape(const rpd_mesh* m, const rpd_sites* sp, const rpd_opts& o, hipStream_t s, int scale,
                      ShapeOut& out, rpd_stats& st) {
  const int ns = sp->n_sites, nt = m->nt;
  const bool dev = (o.flags & RPD_DEVICE_PTRS) != 0;
  // ---- sites
  DBuf site(sizeof(float4) * (size_t)ns);
  DBuf raw;
  const float *sx = sp->sx, *sy = sp->sy, *sz = sp->sz, *sr = sp->sr;
  if (!dev) {
    raw.alloc(sizeof(float) * 4 * (size_t)ns);
    float* r = raw.as<float>();
    hip_check(hipMemcpyAsync(r, sp->sx, sizeof(float) * ns, hipMemcpyHostToDevice, s), "upload");
    hip_check(hipMemcpyAsync(r + ns, sp->sy, sizeof(float) * ns, hipMemcpyHostToDevice, s), "upload");
    hip_check(hipMemcpyAsync(r + 2 * (size_t)ns, sp->sz, sizeof(float) * ns, hipMemcpyHostToDevice, s), "upload");
    hip_check(hipMemcpyAsync(r + 3 * (size_t)ns, sp->sr, sizeof(float) * ns, hipMemcpyHostToDevice, s), "upload");
    sx = r;
    sy = r + ns;
    sz = r + 2 * (size_t)ns;
    sr = r + 3 * (size_t)ns;
  }
  // ---- capacities
  const unsigned capF = pow2_cap((32 * (size_t)ns + 1024) * scale);
  const unsigned capE = pow2_cap((32 * (size_t)ns + 1024) * scale);
  const unsigned capN = pow2_cap((12 * (size_t)nt + 4096) * scale);
  const int rpv_cap = (int)std::min<size_t>((16 * (size_t)ns + 1024) * scale, 1u << 30);
  const int def_cap = (int)std::min<size_t>((4 * (size_t)nt + 4096) * scale, 1u << 30);
  const int piece_cap = (o.flags & RPD_KEEP_PIECES) ? (int)std::min<size_t>((8 * (size_t)nt + 1024) * scale, 1u << 30) : 0;

  DBuf cell_chi(8 * (size_t)ns), cell_geo(32 * (size_t)ns), cell_np(4 * (size_t)ns), cell_b0(4 * (size_t)ns);
  DBuf fkeys(8 * (size_t)capF), face_chi(8 * (size_t)capF), face_b0(4 * (size_t)capF);
  DBuf ekeys(8 * (size_t)capE), edge_chi(8 * (size_t)capE), edge_b0(4 * (size_t)capE);
  DBuf rpv(16 * (size_t)rpv_cap), nkeys(8 * (size_t)capN), node_glue(4 * (size_t)capN), parent(4 * (size_t)capN);
  DBuf deferred(8 * (size_t)def_cap), pieces(sizeof(PieceRec) * (size_t)std::max(piece_cap, 1));
  DBuf counters(8 * NCOUNTERS + 8 * 4), status(16);
  unsigned long long* cnt = counters.as<unsigned long long>();
  unsigned long long* fin_count = cnt + NCOUNTERS;  // [0] faces, [1] edges

  hip_check(launch_fill_u64(cell_chi.as<unsigned long long>(), 0, ns, s), "fill");
  hip_check(launch_fill_u64(cell_geo.as<unsigned long long>(), 0, 4 * (size_t)ns, s), "fill");
  hip_check(launch_fill_i32(cell_np.as<int>(), 0, ns, s), "fill");
  hip_check(launch_fill_i32(cell_b0.as<int>(), 0, ns, s), "fill");
  hip_check(launch_fill_u64(fkeys.as<unsigned long long>(), EMPTY_KEY, capF, s), "fill");
  hip_check(launch_fill_u64(face_chi.as<unsigned long long>(), 0, capF, s), "fill");
  hip_check(launch_fill_i32(face_b0.as<int>(), 0, capF, s), "fill");
  hip_check(launch_fill_u64(ekeys.as<unsigned long long>(), EMPTY_KEY, capE, s), "fill");
  hip_check(launch_fill_u64(edge_chi.as<unsigned long long>(), 0, capE, s), "fill");
  hip_check(launch_fill_i32(edge_b0.as<int>(), 0, capE, s), "fill");
  hip_check(launch_fill_rpv(rpv.as<int4>(), rpv_cap, s), "fill");
  hip_check(launch_fill_u64(nkeys.as<unsigned long long>(), EMPTY_KEY, capN, s), "fill");
  hip_check(launch_fill_i32(node_glue.as<int>(), 0, capN, s), "fill");
  hip_check(launch_fill_u64(cnt, 0, NCOUNTERS + 4, s), "fill");
  hip_check(launch_fill_i32(status.as<int>(), 0, 4, s), "fill");

  ShapeArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nt = nt;
  a.blk = m->blk.as<int>();
  a.nblk = m->nblk;
  a.tp = m->tp.as<float4>();
  a.tn = m->tn.as<int>();
  a.nu = m->nu.as<unsigned>();
  a.L = m->L;
  a.ns = ns;
  a.site = site.as<float4>();
  a.cell_chi = cell_chi.as<long long>();
  a.cell_geo = cell_geo.as<long long>();
  a.cell_np = cell_np.as<int>();
  a.F = HashTab{fkeys.as<unsigned long long>(), capF - 1};
  a.face_chi = face_chi.as<long long>();
  a.E = HashTab{ekeys.as<unsigned long long>(), capE - 1};
  a.edge_chi = edge_chi.as<long long>();
  a.rpv = rpv.as<int4>();
  a.rpv_cap = rpv_cap;
  a.N = HashTab{nkeys.as<unsigned long long>(), capN - 1};
  a.node_glue = node_glue.as<int>();
  a.deferred = deferred.as<int2>();
  a.deferred_cap = def_cap;
  a.pieces = pieces.as<PieceRec>();
  a.piece_cap = piece_cap;
  a.counters = cnt;
  a.status = status.as<int>();
  a.flags = o.flags;
  a.kmax = o.clip_budget > 0 ? std::min(o.clip_budget, KMAX) : KMAX;

  Timing tm((o.flags & RPD_TIMING) != 0);
  tm.mark(0, s);
  hip_check(launch_validate_sites(sx, sy, sz, sr, ns, site.as<float4>(), a.status, s), "validate sites");
  hip_check(launch_clip_fast(a, o.precision, o.block, s), "clip kernel");
  tm.mark(1, s);
  hip_check(launch_clip_slow(a, slow_scratch(), SLOW_THREADS, s), "deferred clip kernel");
  tm.mark(2, s);
  hip_check(launch_glue(a, parent.as<int>(), s), "glue");
  hip_check(launch_count_roots(a, parent.as<int>(), cell_b0.as<int>(), face_b0.as<int>(), edge_b0.as<int>(), s),
            "roots");
  // element lists: sort whole capacities, finalise
  const int maxcap = (int)std::max<unsigned>(std::max(capF, capE), (unsigned)rpv_cap);
  size_t tmpb = sort_tmp_bytes(maxcap);
  DBuf tmp(tmpb), kA(8 * (size_t)maxcap), kB(8 * (size_t)maxcap), kC(8 * (size_t)maxcap), vA(4 * (size_t)maxcap),
      vB(4 * (size_t)maxcap);
  DBuf f_keys(8 * (size_t)capF), f_chi(4 * (size_t)capF), f_b0(4 * (size_t)capF);
  DBuf e_keys(12 * (size_t)capE), e_chi(4 * (size_t)capE), e_b0(4 * (size_t)capE);
  DBuf c_chi(4 * (size_t)ns), c_vol(8 * (size_t)ns), c_cen(24 * (size_t)ns), rpv_sorted(16 * (size_t)rpv_cap);
  hip_check(launch_iota(vA.as<int>(), capF, s), "iota");
  hip_check(sort_pairs_u64(tmp.p, tmpb, fkeys.as<unsigned long long>(), kB.as<unsigned long long>(), vA.as<int>(),
                           vB.as<int>(), capF, s),
            "sort faces");
  hip_check(launch_finalize_faces(kB.as<unsigned long long>(), vB.as<int>(), capF, a.face_chi, face_b0.as<int>(), a.L,
                                  f_keys.as<int>(), f_chi.as<int>(), f_b0.as<int>(), a.status, fin_count + 0, s),
            "finalize faces");
  hip_check(launch_iota(vA.as<int>(), capE, s), "iota");
  hip_check(sort_pairs_u64(tmp.p, tmpb, ekeys.as<unsigned long long>(), kB.as<unsigned long long>(), vA.as<int>(),
                           vB.as<int>(), capE, s),
            "sort edges");
  hip_check(launch_finalize_edges(kB.as<unsigned long long>(), vB.as<int>(), capE, a.edge_chi, edge_b0.as<int>(), a.L,
                                  e_keys.as<int>(), e_chi.as<int>(), e_b0.as<int>(), a.status, fin_count + 1, s),
            "finalize edges");
  hip_check(launch_finalize_cells(ns, a.cell_chi, a.cell_geo, a.cell_np, a.L, c_chi.as<int>(), c_vol.as<double>(),
                                  c_cen.as<double>(), a.status, s),
            "finalize cells");
  hip_check(launch_sort_rpv(a.rpv, rpv_cap, kA.as<unsigned long long>(), kB.as<unsigned long long>(),
                            kC.as<unsigned long long>(), vA.as<int>(), vB.as<int>(), tmp.p, tmpb,
                            rpv_sorted.as<int4>(), s),
            "sort rpv");
  tm.mark(3, s);
  unsigned long long hc[NCOUNTERS + 4];
  int hst = 0;
  hip_check(hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s), "download");
  hip_check(hipMemcpyAsync(&hst, a.status, sizeof(int), hipMemcpyDeviceToHost, s), "download");
  hip_check(hipStreamSynchronize(s), "synchronize");
  if (hst & ST_INVALID) throw Failure{RPD_E_INVALID, "site value off the 2^-20 grid, out of range or not finite"};
  if (hst & ST_DEGENERATE)
    throw Failure{RPD_E_DEGENERATE, "input not in general position (an exact predicate is zero or duplicate sites)"};
  if (hst & ST_TABLE_FULL) return false;
  if (hc[C_DEFER_ITEMS] > (unsigned long long)def_cap || hc[C_RPV] > (unsigned long long)rpv_cap ||
      (piece_cap && hc[C_PIECES] > (unsigned long long)piece_cap))
    return false;
  if (hst & ST_SLOW_CAPACITY)
    throw Failure{RPD_E_NOMEM, "a tet exceeds the large-capacity path (over 1020 candidate sites or 64 vertices)"};
  if (hst & ST_INTERNAL) throw Failure{RPD_E_INTERNAL, "internal consistency check failed (gluing or chi)"};
  const size_t nf = hc[NCOUNTERS + 0], ne = hc[NCOUNTERS + 1], nq = hc[C_RPV];
  out.ns = ns;
  d2h(out.cell_chi, c_chi.p, ns, s);
  d2h(out.cell_b0, cell_b0.p, ns, s);
  d2h(out.vol, c_vol.p, ns, s);
  d2h(out.cen, c_cen.p, 3 * (size_t)ns, s);
  d2h(out.face_keys, f_keys.p, 2 * nf, s);
  d2h(out.face_chi, f_chi.p, nf, s);
  d2h(out.face_b0, f_b0.p, nf, s);
  d2h(out.edge_keys, e_keys.p, 3 * ne, s);
  d2h(out.edge_chi, e_chi.p, ne, s);
  d2h(out.edge_b0, e_b0.p, ne, s);
  d2h(out.rpv_keys, rpv_sorted.p, 4 * nq, s);
  std::vector<PieceRec> prs;
  std::vector<int32_t> perm;
  if (piece_cap) {
    d2h(prs, pieces.p, hc[C_PIECES], s);
    d2h(perm, m->perm.p, nt, s);
  }
  tm.mark(4, s);
  hip_check(hipStreamSynchronize(s), "synchronize");
  out.cell_keys.resize(ns);
  std::iota(out.cell_keys.begin(), out.cell_keys.end(), 0);
  if (piece_cap) {
    std::vector<size_t> ord(prs.size());
    std::iota(ord.begin(), ord.end(), 0);
    for (auto& p : prs) p.t = perm[p.t];
    std::sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
      return prs[x].t != prs[y].t ? prs[x].t < prs[y].t : prs[x].i < prs[y].i;
    });
    for (size_t k : ord) {
      const PieceRec& p = prs[k];
      out.pc_t.push_back(p.t);
      out.pc_i.push_back(p.i);
      out.pc_geo.push_back(p.vol);
      out.pc_geo.push_back(p.mx);
      out.pc_geo.push_back(p.my);
      out.pc_geo.push_back(p.mz);
      out.pc_chi.push_back(p.chi);
    }
  }
  st.n_pairs += (int64_t)hc[C_PAIRS];
  st.n_candidates += (int64_t)hc[C_CAND];
  st.n_deferred += (int64_t)hc[C_DEFER_ITEMS];
  st.n_fp64 += (int64_t)hc[C_FP64];
  st.n_exact += (int64_t)hc[C_EXACT];
  st.n_cells += ns;
  st.n_faces += (int64_t)nf;
  st.n_edges += (int64_t)ne;
  st.n_rpv += (int64_t)nq;
  st.n_glue += (int64_t)hc[C_NODES];
  st.ms_clip += tm.ms(0, 1);
  st.ms_deferred += tm.ms(1, 2);
  st.ms_reduce += tm.ms(2, 3);
  st.ms_total += tm.ms(0, 4);
  return true;
}

}  // namespace rpd

struct rpd_result {
  std::vector<rpd::ShapeOut> shapes;
  rpd_stats stats;
};

using rpd::Failure;

#define RPD_GUARD_BEGIN try {
#define RPD_GUARD_END                          \
  }                                            \
  catch (const Failure& f) {                   \
    rpd::set_error(f.msg);                     \
    return f.code;                             \
  }                                            \
  catch (const std::bad_alloc&) {              \
    rpd::set_error("out of host memory");      \
    return RPD_E_NOMEM;                        \
  }                                            \
  catch (...) {                                \
    rpd::set_error("unexpected C++ exception"); \
    return RPD_E_INTERNAL;                     \
  }

extern "C" {

const char* rpd_version(void) { return "rpd-mi355x 0.1 (gfx950)"; }

const char* rpd_last_error(void) { return rpd::g_error.c_str(); }

rpd_status rpd_mesh_create(const rpd_mesh_desc* desc, uint32_t flags, void* stream, rpd_mesh** out) {
  if (out) *out = nullptr;
  RPD_GUARD_BEGIN
  rpd::set_error("");
  if (!desc || !out) throw Failure{RPD_E_INVALID, "null argument"};
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) throw Failure{RPD_E_DEVICE, "no HIP device"};
  rpd_mesh* m = new rpd_mesh();
  try {
    rpd::mesh_prepare(m, desc, flags, (hipStream_t)stream);
  } catch (...) {
    delete m;
    throw;
  }
  *out = m;
  return RPD_OK;
  RPD_GUARD_END
}

rpd_status rpd_mesh_get_info(const rpd_mesh* m, rpd_mesh_info* info) {
  if (!m || !info) {
    rpd::set_error("null argument");
    return RPD_E_INVALID;
  }
  info->n_verts = m->nv;
  info->n_tets = m->nt;
  info->n_edges = m->n_edges;
  info->n_faces = m->n_faces;
  info->euler = m->euler;
  info->components = m->components;
  info->L = m->L;
  info->volume = m->volume;
  return RPD_OK;
}

void rpd_mesh_free(rpd_mesh* m) { delete m; }

rpd_status rpd_build(const rpd_mesh* const* meshes, const rpd_sites* sites, int32_t n_shapes, const rpd_opts* opts,
                     rpd_result** out) {
  if (out) *out = nullptr;
  RPD_GUARD_BEGIN
  rpd::set_error("");
  if (!meshes || !sites || !out || n_shapes <= 0) throw Failure{RPD_E_INVALID, "null argument or no shape"};
  rpd_opts o;
  std::memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  if (o.precision != RPD_FP32_FALLBACK && o.precision != RPD_FP64) throw Failure{RPD_E_INVALID, "bad precision"};
  if (o.clip_budget != 0 && (o.clip_budget < 4 || o.clip_budget > rpd::KMAX))
    throw Failure{RPD_E_INVALID, "clip_budget must be 0 or in [4, 28]"};
  if (o.block != 0 && o.block != 64 && o.block != 128) throw Failure{RPD_E_INVALID, "block must be 0, 64 or 128"};
  hipStream_t s = (hipStream_t)o.stream;
  rpd_result* r = new rpd_result();
  std::memset(&r->stats, 0, sizeof(r->stats));
  try {
    r->shapes.resize(n_shapes);
    for (int k = 0; k < n_shapes; ++k) {
      const rpd_mesh* m = meshes[k];
      const rpd_sites* sp = &sites[k];
      if (!m) throw Failure{RPD_E_INVALID, "null mesh"};
      if (sp->n_sites <= 0 || sp->n_sites >= (1 << 21) || !sp->sx || !sp->sy || !sp->sz || !sp->sr)
        throw Failure{RPD_E_INVALID, "site count must be in [1, 2^21) with non-null arrays"};
      bool done = false;
      for (int scale = 1; scale <= 16 && !done; scale *= 2) done = rpd::run_shape(m, sp, o, s, scale, r->shapes[k], r->stats);
      if (!done) throw Failure{RPD_E_NOMEM, "result tables kept overflowing"};
    }
  } catch (...) {
    delete r;
    throw;
  }
  *out = r;
  return RPD_OK;
  RPD_GUARD_END
}

static rpd_status shape_check(const rpd_result* r, int32_t shape) {
  if (!r || shape < 0 || shape >= (int32_t)r->shapes.size()) {
    rpd::set_error("bad result handle or shape index");
    return RPD_E_INVALID;
  }
  return RPD_OK;
}

static rpd_status elem_arrays(const rpd_result* r, int32_t shape, int32_t kind, int64_t* n_out, const int32_t** keys,
                              const int32_t** chi, const int32_t** b0) {
  rpd_status e = shape_check(r, shape);
  if (e) return e;
  const rpd::ShapeOut& s = r->shapes[shape];
  if (kind == RPD_CELL) {
    *n_out = s.ns;
    if (keys) *keys = s.cell_keys.data();
    if (chi) *chi = s.cell_chi.data();
    if (b0) *b0 = s.cell_b0.data();
  } else if (kind == RPD_FACE) {
    *n_out = (int64_t)s.face_chi.size();
    if (keys) *keys = s.face_keys.data();
    if (chi) *chi = s.face_chi.data();
    if (b0) *b0 = s.face_b0.data();
  } else if (kind == RPD_EDGE) {
    *n_out = (int64_t)s.edge_chi.size();
    if (keys) *keys = s.edge_keys.data();
    if (chi) *chi = s.edge_chi.data();
    if (b0) *b0 = s.edge_b0.data();
  } else {
    rpd::set_error("bad element kind");
    return RPD_E_INVALID;
  }
  return RPD_OK;
}

rpd_status rpd_euler(const rpd_result* r, int32_t shape, int32_t kind, int64_t* n_out, const int32_t** keys,
                     const int32_t** chi) {
  if (!n_out) return RPD_E_INVALID;
  return elem_arrays(r, shape, kind, n_out, keys, chi, nullptr);
}

rpd_status rpd_components(const rpd_result* r, int32_t shape, int32_t kind, int64_t* n_out, const int32_t** keys,
                          const int32_t** beta0) {
  if (!n_out) return RPD_E_INVALID;
  return elem_arrays(r, shape, kind, n_out, keys, nullptr, beta0);
}

rpd_status rpd_geometry(const rpd_result* r, int32_t shape, const double** vol, const double** centroid) {
  rpd_status e = shape_check(r, shape);
  if (e) return e;
  if (vol) *vol = r->shapes[shape].vol.data();
  if (centroid) *centroid = r->shapes[shape].cen.data();
  return RPD_OK;
}

rpd_status rpd_adjacency(const rpd_result* r, int32_t shape, int32_t kind, int64_t* n_out, const int32_t** keys) {
  rpd_status e = shape_check(r, shape);
  if (e) return e;
  if (!n_out) return RPD_E_INVALID;
  const rpd::ShapeOut& s = r->shapes[shape];
  if (kind == RPD_VERTEX) {
    *n_out = (int64_t)s.rpv_keys.size() / 4;
    if (keys) *keys = s.rpv_keys.data();
    return RPD_OK;
  }
  if (kind == RPD_CELL) {
    rpd::set_error("cells have no adjacency keys");
    return RPD_E_INVALID;
  }
  return elem_arrays(r, shape, kind, n_out, keys, nullptr, nullptr);
}

rpd_status rpd_get_stats(const rpd_result* r, rpd_stats* st) {
  if (!r || !st) return RPD_E_INVALID;
  *st = r->stats;
  return RPD_OK;
}

rpd_status rpd_pieces(const rpd_result* r, int32_t shape, int64_t* n_out, const int32_t** tet, const int32_t** site,
                      const double** vol_moment, const int64_t** chi_num) {
  rpd_status e = shape_check(r, shape);
  if (e) return e;
  if (!n_out) return RPD_E_INVALID;
  const rpd::ShapeOut& s = r->shapes[shape];
  *n_out = (int64_t)s.pc_t.size();
  if (tet) *tet = s.pc_t.data();
  if (site) *site = s.pc_i.data();
  if (vol_moment) *vol_moment = s.pc_geo.data();
  if (chi_num) *chi_num = s.pc_chi.data();
  return RPD_OK;
}

void rpd_free(rpd_result* r) { delete r; }

}  // extern "C"
