// C ABI of librpd (declared in include/rpd.h): argument checking, buffer management, kernel sequencing on the
// caller's stream, and the host copies of the results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "rpd.h"
#include "rpd_host.h"
#include "rpd_launch.h"

namespace rpd {

static thread_local char g_error[512];
void set_error(const char* msg) {
  size_t k = 0;
  for (; msg[k] && k + 1 < sizeof(g_error); ++k) g_error[k] = msg[k];
  g_error[k] = 0;
}

// ---- caching allocator
static std::mutex g_pool_mu;
static std::map<std::pair<int, size_t>, std::vector<void*>> g_pool;

void* pool_alloc(size_t bytes, size_t* cls_bytes, int* device) {
  size_t c = 256;
  while (c < bytes) c <<= 1;
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  *device = dev;
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

void pool_free(void* p, size_t cls_bytes, int device) {
  std::lock_guard<std::mutex> g(g_pool_mu);
  g_pool[{device, cls_bytes}].push_back(p);
}

static unsigned pow2_cap(size_t n) {
  size_t c = 1024;
  while (c < n) c <<= 1;
  if (c > (1u << 31)) throw Failure{RPD_E_NOMEM, "table capacity above 2^31"};
  return (unsigned)c;
}

// Waves of the large-capacity kernel: one deferred item per wave at a time; each wave owns a private scratch
// region of slow_scratch_bytes(1) (about 240 KB), allocated with the call's other buffers.
static int slow_waves(long long nt) { return (int)std::max<long long>(64, std::min<long long>(2048, nt / 16)); }

struct HostPinned;

// A result array: its own storage, or a view into the call's downloaded (pinned) buffer that the result keeps.
template <typename T>
struct Arr {
  std::vector<T> own;
  const T* ext = nullptr;
  size_t n_ext = 0;
  bool is_view = false;
  const T* data() const { return is_view ? ext : own.data(); }
  size_t size() const { return is_view ? n_ext : own.size(); }
  const T* begin() const { return data(); }
  const T* end() const { return data() + size(); }
  void view(const T* p, size_t n) {
    own.clear();
    ext = p;
    n_ext = n;
    is_view = true;
  }
  std::vector<T>& owned() {
    is_view = false;
    return own;
  }
};

struct ShapeOut {
  int ns = 0;
  std::shared_ptr<HostPinned> hold;  // the downloaded buffer the views point into
  Arr<int32_t> cell_keys, cell_chi, cell_b0;
  Arr<double> vol, cen;
  Arr<int32_t> face_keys, face_chi, face_b0;
  Arr<int32_t> edge_keys, edge_chi, edge_b0;
  Arr<double> edge_len, edge_alpha;
  Arr<int32_t> rpv_keys;
  std::vector<int32_t> pc_t, pc_i;
  std::vector<double> pc_geo;
  std::vector<int64_t> pc_chi;
  // per-piece element terms by kind (cell, face, edge, RPV): caller tet, kind site ids, numerator, gluing bits
  std::vector<int32_t> tm_t[4], tm_s[4], tm_glue[4];
  std::vector<int64_t> tm_num[4];
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
    hip_check(hipEventSynchronize(ev[b]), "hipEventSynchronize");
    hip_check(hipEventElapsedTime(&x, ev[a], ev[b]), "hipEventElapsedTime");
    return x;
  }
};

template <class T>
static void d2h(std::vector<T>& v, const void* src, size_t n, hipStream_t s) {
  v.resize(n);
  if (n) hip_check(hipMemcpyAsync(v.data(), src, sizeof(T) * n, hipMemcpyDeviceToHost, s), "download");
}

// vertex slots per piece of the FP32 fast kernel: 12 only where asked for with 64 threads, else 16
static int fast_slots(const rpd_opts& o) {
  return (o.precision == RPD_FP32_FALLBACK && (o.block == 0 || o.block == 64) && o.slots == 12) ? 12 : 16;
}

// ---------------------------------------------------------------------------------------------------------------
// Device state of one computation: tables, accumulators, counters. Used once by rpd_build and kept across rounds
// by a session.
// ---------------------------------------------------------------------------------------------------------------
struct DeviceState {
  int nsh = 0, ns_cap = 0;
  long long nt_tot = 0;
  unsigned capF = 0, capE = 0, capQ = 0, capN = 0;
  int def_cap = 0, piece_cap = 0, term_cap = 0, list_cap = 0, big_cap = 0;
  DBuf site, status, cell_chi, cell_geo, cell_np, cell_b0;
  DBuf fkeys, face_chi, face_np, face_b0, ekeys, edge_chi, edge_np, edge_len, edge_b0, qkeys, rpv_cnt;
  DBuf nodes, glist, gseg, clist, cseg, bigp, deferred, deferred2, dlist, pieces, terms, counters, tetU, slow, touch, removed;
  int waves = 0;

  unsigned long long* cnt() const { return counters.as<unsigned long long>(); }
  unsigned long long* fin_count() const { return cnt() + NCOUNTERS; }  // [0] faces, [1] edges
  unsigned long long* stat() const { return cnt() + NCOUNTERS + 8; }  // [NSPREAD][NCOUNTERS]
  // totals of every counter: the cursor and the sum of its spread copies (synchronises the stream)
  // counter totals (cursors, list counts and the sums of the spread statistics) and the status word, in one
  // round trip through pinned memory
  void totals(unsigned long long* out, hipStream_t s, int* status_out = nullptr) const;
  size_t touch_words() const { return ((size_t)ns_cap + capF + capE + 3) / 4; }

  void alloc(int n_shapes, int ns, long long nt, int scale, bool keep_pieces, bool keep_U, int slots) {
    nsh = n_shapes;
    ns_cap = ns;
    nt_tot = nt;
    capF = pow2_cap((32 * (size_t)ns + 1024) * scale);
    capE = pow2_cap((32 * (size_t)ns + 1024) * scale);
    capQ = pow2_cap((16 * (size_t)ns + 1024) * scale);
    // element pieces: 12 slots per tet keeps the probe chains of the emission's inserts short; past 2^23 slots
    // the table scans of the gluing pass cost more than that saves, so large meshes get 6
    capN = pow2_cap((12 * (size_t)nt + 4096) * scale);
    if (capN > (1u << 23)) capN = std::max(1u << 23, pow2_cap((6 * (size_t)nt + 4096) * scale));
    def_cap = (int)std::min<size_t>((4 * (size_t)nt + 4096) * scale, 1u << 30);
    piece_cap = keep_pieces ? (int)std::min<size_t>((8 * (size_t)nt + 1024) * scale, 1u << 30) : 0;
    term_cap = keep_pieces ? (int)std::min<size_t>((24 * (size_t)nt + 4096) * scale, 1u << 30) : 0;
    site.alloc(sizeof(float4) * (size_t)ns);
    status.alloc(16);
    cell_chi.alloc(8 * (size_t)ns);
    cell_geo.alloc(64 * (size_t)ns);  // volume and first moment: four 128-bit accumulators per site
    cell_np.alloc(4 * (size_t)ns);
    cell_b0.alloc(4 * (size_t)ns);
    fkeys.alloc(8 * (size_t)capF);
    face_chi.alloc(8 * (size_t)capF);
    face_np.alloc(4 * (size_t)capF);
    face_b0.alloc(4 * (size_t)capF);
    ekeys.alloc(8 * (size_t)capE);
    edge_chi.alloc(8 * (size_t)capE);
    edge_np.alloc(4 * (size_t)capE);
    edge_len.alloc(8 * (size_t)capE);
    edge_b0.alloc(4 * (size_t)capE);
    qkeys.alloc(8 * (size_t)capQ);
    rpv_cnt.alloc(4 * (size_t)capQ);
    nodes.alloc(sizeof(NodeRec) * (size_t)capN);
    glist.alloc(sizeof(int) * (size_t)capN);
    gseg.alloc(sizeof(int) * (size_t)capN / 256);  // the gluing list's segments
    deferred.alloc(16 * (size_t)def_cap);
    deferred2.alloc(16 * (size_t)(def_cap / 4 + 1024));
    // candidate lists of deferred tets and pieces (a few per cent of the tets on the heaviest workloads)
    list_cap = (int)std::min<size_t>((nt / 8 + 4096) * (size_t)scale, (1u << 25) - 1);
    dlist.alloc(sizeof(int) * KRAW * (size_t)list_cap);
    // pieces over the fast kernel's vertex slots: about 1 in 10^4 on the benchmark shapes with 16 slots, up to 1 in
    // 10^2 with 12; an incremental session gets room for four times as many per pass as a build (its pool must
    // never run out)
    const long long per_big = slots == 12 ? (keep_U ? 8 : 32) : (keep_U ? 64 : 256);
    big_cap = (int)std::min<size_t>((nt / per_big + 1024) * (size_t)scale, 1u << 20);
    bigp.alloc(BIG_BYTES * (size_t)big_cap);
    pieces.alloc(sizeof(PieceRec) * (size_t)std::max(piece_cap, 1));
    terms.alloc(sizeof(TermRec) * (size_t)std::max(term_cap, 1));
    counters.alloc(8 * (NCOUNTERS + 8 + (size_t)NSPREAD * NCOUNTERS));
    if (keep_U) {  // incremental updates: U_t per tet, the touched-element flags, the removed-piece tags
      tetU.alloc(8 * (size_t)std::max<long long>(nt, 1));
      touch.alloc(touch_words() * 4);
      removed.alloc(4 * (size_t)capN);
      clist.alloc(sizeof(int) * (size_t)capN);  // the live cell pieces, for the rounds' selection scans
      cseg.alloc(sizeof(int) * (size_t)capN / 256);
    }
    waves = slow_waves(nt);
    slow.alloc(slow_scratch_bytes(waves));
  }

  void clear(hipStream_t s) {  // one launch for every accumulator and table
    const size_t ns = (size_t)ns_cap;
    FillList L{};
    L.add(status.p, 0, 4, 4);
    L.add(cell_chi.p, 0, ns, 8);
    L.add(cell_geo.p, 0, 8 * ns, 8);
    L.add(cell_np.p, 0, ns, 4);
    L.add(fkeys.p, EMPTY_KEY, capF, 8);
    L.add(face_chi.p, 0, capF, 8);
    L.add(face_np.p, 0, capF, 4);
    L.add(ekeys.p, EMPTY_KEY, capE, 8);
    L.add(edge_chi.p, 0, capE, 8);
    L.add(edge_np.p, 0, capE, 4);
    L.add(edge_len.p, 0, capE, 8);
    L.add(qkeys.p, EMPTY_KEY, capQ, 8);
    L.add(rpv_cnt.p, 0, capQ, 4);
    L.add(nodes.p, EMPTY_KEY, capN, 16, 0ull);  // key EMPTY, state 0, parent 0
    L.add(cnt(), 0, NCOUNTERS + 8 + (size_t)NSPREAD * NCOUNTERS, 8);
    if (touch.p) L.add(touch.p, 0, touch_words(), 4);
    if (removed.p) L.add(removed.p, 0, capN, 4);
    hip_check(launch_fill_multi(L, s), "fill");
  }

  // the touched-element flags for an incremental pass
  void set_touch(ShapeArgs& a) const {
    unsigned char* t = touch.as<unsigned char>();
    a.touch_cell = t;
    a.touch_face = t + ns_cap;
    a.touch_edge = t + ns_cap + capF;
    a.removed = removed.as<unsigned short>();
  }

  ShapeArgs args(const ShapeDesc* shapes, const int2* items, int nitems, unsigned flags, int kmax) const {
    ShapeArgs a;
    std::memset(&a, 0, sizeof(a));
    a.shapes = shapes;
    a.nshapes = nsh;
    a.items = items;
    a.nitems = nitems;
    a.ns = ns_cap;
    a.site = site.as<float4>();
    a.cell_chi = cell_chi.as<long long>();
    a.cell_geo = cell_geo.as<long long>();
    a.cell_np = cell_np.as<int>();
    a.F = HashTab{fkeys.as<unsigned long long>(), capF - 1};
    a.face_chi = face_chi.as<long long>();
    a.face_np = face_np.as<int>();
    a.E = HashTab{ekeys.as<unsigned long long>(), capE - 1};
    a.edge_chi = edge_chi.as<long long>();
    a.edge_np = edge_np.as<int>();
    a.edge_len = edge_len.as<long long>();
    a.Q = HashTab{qkeys.as<unsigned long long>(), capQ - 1};
    a.rpv_cnt = rpv_cnt.as<int>();
    a.N = NodeTab{nodes.as<NodeRec>(), capN - 1};
    a.tet_U = tetU.p ? tetU.as<double>() : nullptr;
    a.deferred = deferred.as<int4>();
    a.deferred_cap = def_cap;
    a.deferred2 = deferred2.as<int4>();
    a.deferred2_cap = def_cap / 4 + 1024;
    a.deferred_list = dlist.as<int>();
    a.list_cap = list_cap;
    a.big = bigp.as<unsigned char>();
    a.big_cap = big_cap;
    a.pieces = pieces.as<PieceRec>();
    a.piece_cap = piece_cap;
    a.terms = terms.as<TermRec>();
    a.term_cap = term_cap;
    a.counters = cnt();
    a.stats = stat();
    a.status = status.as<int>();
    a.flags = flags;
    a.kmax = kmax;
    return a;
  }

  // components of every live element piece: fresh union-find and root counts
  // (with a.touch_* set: of the touched elements only, then the flags are cleared)
  void components(const ShapeArgs& a, hipStream_t s) {
    if (a.touch_cell) {
      hip_check(launch_clear_touched_b0(a.touch_cell, cell_b0.as<int>(), (size_t)ns_cap, s), "clear");
      hip_check(launch_clear_touched_b0(a.touch_face, face_b0.as<int>(), capF, s), "clear");
      hip_check(launch_clear_touched_b0(a.touch_edge, edge_b0.as<int>(), capE, s), "clear");
    } else {
      FillList L{};
      L.add(cell_b0.p, 0, (size_t)ns_cap, 4);
      L.add(face_b0.p, 0, capF, 4);
      L.add(edge_b0.p, 0, capE, 4);
      L.add_stats_zero(stat(), NSPREAD, C_NODES, 1, C_GLUE_BITS, 2);
      hip_check(launch_fill_multi(L, s), "fill");
    }
    if (a.touch_cell) hip_check(launch_zero_stats(stat(), C_NODES, 1, C_GLUE_BITS, 2, s), "fill");
    hip_check(launch_glue(a, glist.as<int>(), gseg.as<int>(), clist.as<int>(), cseg.as<int>(), s), "glue");
    hip_check(launch_count_roots(a, glist.as<int>(), gseg.as<int>(), cell_b0.as<int>(), face_b0.as<int>(),
                                 edge_b0.as<int>(), s),
              "roots");
    if (a.touch_cell) hip_check(launch_fill_i32(touch.as<int>(), 0, touch_words(), s), "fill");
  }
};

static rpd_status status_error(int hst) {
  if (hst & ST_INVALID) throw Failure{RPD_E_INVALID, "site value off the 2^-20 grid, out of range or not finite"};
  if (hst & ST_DEGENERATE)
    throw Failure{RPD_E_DEGENERATE, "three clipping planes without a single meet point"};
  if (hst & ST_SLOW_CAPACITY)
    throw Failure{RPD_E_NOMEM, "a tet exceeds the large-capacity path (over 1020 candidate sites or 64 vertices)"};
  if (hst & ST_INTERNAL) throw Failure{RPD_E_INTERNAL, "internal consistency check failed (gluing or chi)"};
  return RPD_OK;
}

// Pinned host staging for the result download (one copy per call), pooled like device memory.
static std::mutex g_pin_mu;
static std::map<size_t, std::vector<void*>> g_pin_pool;

struct HostPinned {
  void* p = nullptr;
  size_t bytes = 0;
  explicit HostPinned(size_t n) {
    size_t c = 4096;
    while (c < n) c <<= 1;
    bytes = c;
    {
      std::lock_guard<std::mutex> g(g_pin_mu);
      auto& v = g_pin_pool[c];
      if (!v.empty()) {
        p = v.back();
        v.pop_back();
        return;
      }
    }
    hip_check(hipHostMalloc(&p, c, hipHostMallocDefault), "hipHostMalloc");
  }
  ~HostPinned() {
    std::lock_guard<std::mutex> g(g_pin_mu);
    g_pin_pool[bytes].push_back(p);
  }
  HostPinned(const HostPinned&) = delete;
  HostPinned& operator=(const HostPinned&) = delete;
};

void DeviceState::totals(unsigned long long* out, hipStream_t s, int* status_out) const {
  const size_t n = NCOUNTERS + 8 + (size_t)NSPREAD * NCOUNTERS;
  HostPinned h(8 * n + 16);
  unsigned long long* hv = (unsigned long long*)h.p;
  hip_check(hipMemcpyAsync(hv, cnt(), 8 * n, hipMemcpyDeviceToHost, s), "download");
  if (status_out) hip_check(hipMemcpyAsync(hv + n, status.p, sizeof(int), hipMemcpyDeviceToHost, s), "download");
  hip_check(hipStreamSynchronize(s), "synchronize");
  for (int c = 0; c < NCOUNTERS + 8; ++c) out[c] = hv[c];
  for (int k = 0; k < NSPREAD; ++k)
    for (int c = 0; c < NCOUNTERS; ++c) out[c] += hv[NCOUNTERS + 8 + (size_t)k * NCOUNTERS + c];
  if (status_out) *status_out = *(const int*)(hv + n);
}

// Bytes of the result download of the last call per (sites, shapes, table sizes): the next such call queues the copy
// of that prefix (plus an eighth) before the host waits for the counts, so that a call with about as many elements
// takes one host round trip instead of two; a larger result is downloaded again after the counts.
static std::mutex g_spec_mu;
static std::map<std::tuple<int, int, unsigned, unsigned, unsigned>, size_t> g_spec;

// Sorted element lists of the current state, copied to the host and split per shape. Returns false when a table
// overflowed (the caller retries with larger tables). Live entries are compacted first and the counts read back,
// so that only they are sorted and downloaded.
static bool collect(DeviceState& D, const std::vector<ShapeDesc>& hd, const ShapeDesc* dshapes,
                    const rpd_mesh* const* meshes, hipStream_t s, Timing& tm, std::vector<ShapeOut>& outs,
                    rpd_stats& st) {
  const int nsh = (int)hd.size();
  int ns = 0;
  for (const auto& d : hd) ns = std::max(ns, d.site_off + d.ns);
  const unsigned capF = D.capF, capE = D.capE, capQ = D.capQ;
  unsigned long long* fin = D.fin_count();  // [0] faces, [1] edges, [2] RPVs
  DBuf fk(8 * (size_t)capF), fsl(4 * (size_t)capF), ek(8 * (size_t)capE), esl(4 * (size_t)capE),
      rq(16 * (size_t)capQ);
  // the list counts were zeroed with the other counters when the state was cleared; an incremental session collects
  // again and again from one state
  if (D.touch.p) hip_check(launch_fill_u64(fin, 0, 3, s), "fill");
  // the row sort's per-row counts and cursors (3 (ns + 1) and 3 ns ints), cleared, and its tile sums
  const size_t n_rowc = 3 * ((size_t)ns + 1) + 3 * (size_t)std::max(ns, 1);
  DBuf rowc(4 * (n_rowc + 3 * (size_t)row_tiles(std::max(ns, 1))));
  {
    CompactLists J;
    J.live[0] = {D.fkeys.as<unsigned long long>(), D.face_np.as<int>(), capF, 0, fk.as<unsigned long long>(),
                 fsl.as<int>(), fin + 0};
    J.live[1] = {D.ekeys.as<unsigned long long>(), D.edge_np.as<int>(), capE, 0, ek.as<unsigned long long>(),
                 esl.as<int>(), fin + 1};
    J.Q = HashTab{D.qkeys.as<unsigned long long>(), capQ - 1};
    J.rpv_cnt = D.rpv_cnt.as<int>();
    J.ekeys = D.ekeys.as<unsigned long long>();
    J.rpv_cpt = 0;
    J.rpv_out = rq.as<int4>();
    J.rpv_count = fin + 2;
    J.zero = rowc.as<int>();  // the row sort's counters, cleared in the same launch
    J.n_zero = n_rowc;
    hip_check(launch_compact_lists(J, s), "live faces, edges and rpvs");
  }
  const HashTab F{D.fkeys.as<unsigned long long>(), capF - 1}, E{D.ekeys.as<unsigned long long>(), capE - 1};
  const size_t ncap = std::max<size_t>(std::max(capF, capE), capQ);
  unsigned long long hc[NCOUNTERS + 8];
  int hst = 0;
  // the counters, status and live counts: a false return (a table or buffer overflowed) has the caller retry
  auto check_totals = [&]() {
    D.totals(hc, s, &hst);
    if (hst & ST_TABLE_FULL) return false;
    if (hc[C_DEFER_ITEMS] > (unsigned long long)D.def_cap || hc[C_LISTS] > (unsigned long long)D.list_cap ||
        (D.piece_cap &&
         (hc[C_PIECES] > (unsigned long long)D.piece_cap || hc[C_TERMS] > (unsigned long long)D.term_cap)))
      return false;
    status_error(hst);
    return true;
  };
  // one device buffer carries everything to the host (OutLayout); the kernels place their output from the live
  // counts in device memory
  DBuf out;
  OutDesc od{nullptr, fin, ns, nsh};
  size_t nf = 0, ne = 0, nq = 0;
  const auto spec_key = std::make_tuple(ns, nsh, capF, capE, capQ);
  std::shared_ptr<HostPinned> host;  // kept by the result (its arrays point into it)
  size_t spec = 0;                   // bytes downloaded before the counts were known
  {
    // the lists are sorted by rows of their first site and slots are looked up again by key; the whole sequence is
    // queued before the host waits for the counts (the buffer is sized for full tables)
    out.alloc(out_layout(ns, nsh, capF, capE, capQ).bytes);
    od.base = out.as<unsigned char>();
    DBuf kq(8 * (size_t)capQ), t0(8 * (size_t)capF), t1(8 * (size_t)capE), t2(8 * (size_t)capQ),
        qrow(4 * (size_t)capQ);
    unsigned long long* const keys[3] = {fk.as<unsigned long long>(), ek.as<unsigned long long>(),
                                         kq.as<unsigned long long>()};
    unsigned long long* const tmps[3] = {t0.as<unsigned long long>(), t1.as<unsigned long long>(),
                                         t2.as<unsigned long long>()};
    const size_t caps[3] = {capF, capE, capQ};
    const int shifts[3] = {32, 42, 0};  // RPVs: rows carried beside the keys
    hip_check(launch_row_sort(keys, tmps, fin, caps, shifts, std::max(ns, 1), rowc.as<int>(),
                              rowc.as<int>() + 3 * ((size_t)ns + 1), rq.as<int4>(), qrow.as<int>(),
                              rowc.as<int>() + n_rowc, s),
              "sort lists");
    FinalizeRows R;
    R.fkeys = fk.as<unsigned long long>();
    R.ekeys = ek.as<unsigned long long>();
    R.qkeys = kq.as<unsigned long long>();
    R.qrows = qrow.as<int>();
    R.F = F;
    R.E = E;
    R.face_chi = D.face_chi.as<long long>();
    R.edge_chi = D.edge_chi.as<long long>();
    R.edge_len = D.edge_len.as<long long>();
    R.cell_chi = D.cell_chi.as<long long>();
    R.cell_geo = D.cell_geo.as<long long>();
    R.face_b0 = D.face_b0.as<int>();
    R.edge_b0 = D.edge_b0.as<int>();
    R.cell_np = D.cell_np.as<int>();
    R.cell_b0 = D.cell_b0.as<int>();
    R.site = D.site.as<float4>();
    R.ns = ns;
    hip_check(launch_finalize_rows(R, ncap, od, dshapes, nsh, D.status.as<int>(), s), "finalize lists and cells");
    if (nsh > 1) hip_check(launch_localize_lists(od, ncap, dshapes, nsh, s), "localize lists");
    tm.mark(3, s);
    if (!D.piece_cap) {
      std::lock_guard<std::mutex> g(g_spec_mu);
      auto it = g_spec.find(spec_key);
      if (it != g_spec.end()) spec = std::min(out.bytes, it->second + it->second / 8 + 4096);
    }
    if (spec) {
      host = std::make_shared<HostPinned>(spec);
      hip_check(hipMemcpyAsync(host->p, od.base, spec, hipMemcpyDeviceToHost, s), "download");
      tm.mark(4, s);  // complete once the counts have arrived
    }
    if (!check_totals()) return false;  // the prefix has arrived too
    nf = hc[NCOUNTERS + 0];
    ne = hc[NCOUNTERS + 1];
    nq = hc[NCOUNTERS + 2];
  }
  const OutLayout L = out_layout(ns, nsh, nf, ne, nq);
  const size_t out_bytes = L.bytes;
  if (!D.piece_cap) {
    std::lock_guard<std::mutex> g(g_spec_mu);
    g_spec[spec_key] = out_bytes;
  }
  const bool have = spec > 0 && out_bytes <= spec;
  if (!have) host = std::make_shared<HostPinned>(out_bytes + 16);
  unsigned char* hb = (unsigned char*)host->p;
  if (!have) {
    hip_check(hipMemcpyAsync(hb, od.base, out_bytes, hipMemcpyDeviceToHost, s), "download");
    hip_check(hipMemcpyAsync(hb + out_bytes, D.status.p, sizeof(int), hipMemcpyDeviceToHost, s), "download");
  }
  std::vector<PieceRec> prs;
  if (D.piece_cap) d2h(prs, D.pieces.p, hc[C_PIECES], s);
  std::vector<TermRec> trs;
  if (D.piece_cap) d2h(trs, D.terms.p, hc[C_TERMS], s);
  if (!have) tm.mark(4, s);
  if (!have) {
    hip_check(hipStreamSynchronize(s), "synchronize");
    status_error(*(int*)(hb + out_bytes));
  }
  const int* all_rpv = (const int*)(hb + L.rpv);
  const int* all_cchi = (const int*)(hb + L.cchi);
  const int* all_cb0 = (const int*)(hb + L.cb0);
  const int* all_fk = (const int*)(hb + L.fk);
  const int* all_fchi = (const int*)(hb + L.fchi);
  const int* all_fb0 = (const int*)(hb + L.fb0);
  const int* all_ek = (const int*)(hb + L.ek);
  const int* all_echi = (const int*)(hb + L.echi);
  const int* all_eb0 = (const int*)(hb + L.eb0);
  const double* all_vol = (const double*)(hb + L.vol);
  const double* all_cen = (const double*)(hb + L.cen);
  const double* all_elen = (const double*)(hb + L.elen);
  const double* all_ealpha = (const double*)(hb + L.ealpha);
  // ---- split per shape (element lists are sorted by batch-global keys, so each shape is one contiguous run; the
  //      device found the runs and turned the keys into shape-local site ids)
  std::vector<size_t> run[3];
  {
    const size_t tot[3] = {nf, ne, nq};
    const int* starts = (const int*)(hb + L.start);
    for (int y = 0; y < 3; ++y) {
      run[y].assign((size_t)nsh + 1, tot[y]);
      if (nsh == 1) run[y][0] = 0;
      for (int k = nsh - 1; k >= 0 && nsh > 1; --k) {
        const int v = starts[(size_t)y * nsh + k];
        run[y][k] = v >= 0 ? (size_t)v : run[y][k + 1];  // a shape without elements: an empty run
      }
    }
  }
  for (int k = 0; k < nsh; ++k) {
    ShapeOut& out = outs[k];
    const int off = hd[k].site_off, n = hd[k].ns;
    out.ns = n;
    out.hold = host;
    out.cell_chi.view(all_cchi + off, n);
    out.cell_b0.view(all_cb0 + off, n);
    out.vol.view(all_vol + off, n);
    out.cen.view(all_cen + 3 * (size_t)off, 3 * (size_t)n);
    std::vector<int32_t>& ck = out.cell_keys.owned();
    ck.resize(n);
    std::iota(ck.begin(), ck.end(), 0);
    const size_t fpos = run[0][k], fend = run[0][k + 1], epos = run[1][k], eend = run[1][k + 1], qpos = run[2][k],
                 qend = run[2][k + 1];
    out.face_keys.view(all_fk + 2 * fpos, 2 * (fend - fpos));
    out.face_chi.view(all_fchi + fpos, fend - fpos);
    out.face_b0.view(all_fb0 + fpos, fend - fpos);
    out.edge_keys.view(all_ek + 3 * epos, 3 * (eend - epos));
    out.edge_chi.view(all_echi + epos, eend - epos);
    out.edge_b0.view(all_eb0 + epos, eend - epos);
    out.edge_len.view(all_elen + epos, eend - epos);
    out.edge_alpha.view(all_ealpha + epos, eend - epos);
    out.rpv_keys.view(all_rpv + 4 * qpos, 4 * (qend - qpos));
    out.pc_t.clear();
    out.pc_i.clear();
    out.pc_geo.clear();
    out.pc_chi.clear();
    for (int q = 0; q < 4; ++q) {
      out.tm_t[q].clear();
      out.tm_s[q].clear();
      out.tm_num[q].clear();
      out.tm_glue[q].clear();
    }
  }
  if (D.piece_cap) {
    std::vector<std::vector<int32_t>> perms(nsh);
    std::vector<std::vector<size_t>> per_shape(nsh);
    std::vector<std::vector<size_t>> terms_of(nsh);
    auto shape_of = [&](long long t) {
      int lo = 0, hi = nsh - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (hd[mid].tet_off <= t) lo = mid;
        else hi = mid - 1;
      }
      return lo;
    };
    for (size_t q = 0; q < prs.size(); ++q) per_shape[shape_of(prs[q].t)].push_back(q);
    for (size_t q = 0; q < trs.size(); ++q) terms_of[shape_of(trs[q].t)].push_back(q);
    for (int k = 0; k < nsh; ++k) {
      if (per_shape[k].empty()) continue;
      d2h(perms[k], meshes[k]->perm.p, meshes[k]->nt, s);
      hip_check(hipStreamSynchronize(s), "synchronize");
      auto& idx = per_shape[k];
      auto tt = [&](size_t q) { return perms[k][prs[q].t - (int)hd[k].tet_off]; };
      std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
        return tt(x) != tt(y) ? tt(x) < tt(y) : prs[x].i < prs[y].i;
      });
      ShapeOut& out = outs[k];
      // element terms of the shape's pieces, by kind, ordered by (caller tet, site ids)
      std::vector<size_t>& tix = terms_of[k];
      auto tkey = [&](size_t q) {
        const TermRec& r = trs[q];
        return std::make_tuple(r.kind, perms[k][r.t - (int)hd[k].tet_off], r.i, r.j, r.k, r.l);
      };
      std::sort(tix.begin(), tix.end(), [&](size_t x, size_t y) { return tkey(x) < tkey(y); });
      for (size_t q : tix) {
        const TermRec& r = trs[q];
        const int kind = r.kind, off = hd[k].site_off;
        out.tm_t[kind - 1].push_back(perms[k][r.t - (int)hd[k].tet_off]);
        const int ids[4] = {r.i, r.j, r.k, r.l};
        for (int c = 0; c < kind; ++c) out.tm_s[kind - 1].push_back(ids[c] - off);
        out.tm_num[kind - 1].push_back(r.num);
        out.tm_glue[kind - 1].push_back(r.glue);
      }
      for (size_t q : idx) {
        const PieceRec& p = prs[q];
        out.pc_t.push_back(tt(q));
        out.pc_i.push_back(p.i - hd[k].site_off);
        out.pc_geo.push_back(p.vol);
        out.pc_geo.push_back(p.mx);
        out.pc_geo.push_back(p.my);
        out.pc_geo.push_back(p.mz);
        out.pc_chi.push_back(p.chi);
      }
    }
  }
  st.n_pairs = (int64_t)hc[C_PAIRS];
  st.n_candidates = (int64_t)hc[C_CAND];
  st.n_deferred = (int64_t)hc[C_DEFER_ITEMS];
  st.n_fp64 = (int64_t)hc[C_FP64];
  st.n_exact = (int64_t)hc[C_EXACT];
  st.n_cells = ns;
  st.n_faces = (int64_t)nf;
  st.n_edges = (int64_t)ne;
  st.n_rpv = (int64_t)nq;
  st.n_glue = (int64_t)hc[C_NODES];
  st.n_defer_block = (int64_t)hc[C_DEFER_BLOCK];
  st.n_defer_kmax = (int64_t)hc[C_DEFER_KMAX];
  st.n_defer_clip = (int64_t)hc[C_DEFER_CLIP];
  st.n_split = (int64_t)hc[C_SPLIT];
  st.n_big = (int64_t)hc[C_BIG];
  return true;
}

static std::vector<ShapeDesc> shape_table(const rpd_mesh* const* meshes, const int* nsites, int nsh, long long* ns_tot,
                                          long long* nt_tot) {
  std::vector<ShapeDesc> hd(nsh);
  *ns_tot = 0;
  *nt_tot = 0;
  for (int k = 0; k < nsh; ++k) {
    const rpd_mesh* m = meshes[k];
    ShapeDesc& d = hd[k];
    d.tp = m->tp.as<float4>();
    d.tf = m->tf.as<double4>();
    d.tn = m->tn.as<int>();
    d.nu = m->nu.as<unsigned>();
    d.blk = m->blk.as<int>();
    d.nt = m->nt;
    d.nblk = m->nblk;
    d.L = m->L;
    d.site_off = (int)*ns_tot;
    d.ns = nsites[k];
    d.tet_off = *nt_tot;
    d.sign = +1;
    d.pad = 0;
    *ns_tot += nsites[k];
    *nt_tot += m->nt;
  }
  for (int k = 0; k < nsh; ++k)
    if (hd[k].nblk >= (1 << ITEM_PART_SHIFT)) throw Failure{RPD_E_INVALID, "mesh with 2^20 or more workgroup blocks"};
  if (*ns_tot >= (1 << 21)) throw Failure{RPD_E_INVALID, "more than 2^21 - 1 sites in one call"};
  if (*nt_tot >= (1ll << 31)) throw Failure{RPD_E_INVALID, "more than 2^31 - 1 tets in one call"};
  return hd;
}

// (shape, block) work items, heaviest first. The hardware dispatcher hands workgroups to compute units in grid
// order as they free up, so a heavy item dispatched late sets the kernel's tail. The cost of an item is its
// fast-kernel time in the last build on the same mesh when every mesh of the call has one (and
// RPD_ESTIMATED_ORDER is not set), else the estimate shape sites x block tets (the box filter scans every site of the shape; clipping grows with the tets).
// Ties keep the shapes' order and the blocks' Morton order. The order never changes a result.
static std::vector<int2> work_items(const std::vector<ShapeDesc>& hd, const rpd_mesh* const* meshes,
                                    unsigned flags) {
  const int nsh = (int)hd.size();
  std::vector<int2> items;
  std::vector<unsigned long long> cost;
  bool learned = (flags & RPD_ESTIMATED_ORDER) == 0;
  for (int k = 0; k < nsh && learned; ++k) {
    rpd_mesh* m = const_cast<rpd_mesh*>(meshes[k]);
    std::lock_guard<std::mutex> g(m->cost_mu);
    learned = (int)m->blk_cost.size() == hd[k].nblk;
  }
  for (int k = 0; k < nsh; ++k) {
    rpd_mesh* m = const_cast<rpd_mesh*>(meshes[k]);
    std::unique_lock<std::mutex> g(m->cost_mu, std::defer_lock);
    if (learned) g.lock();
    for (int b = 0; b < hd[k].nblk; ++b) {
      items.push_back(make_int2(k, b));
      cost.push_back(learned ? (unsigned long long)m->blk_cost[b]
                             : (unsigned long long)hd[k].ns * (unsigned long long)(m->hblk[b + 1] - m->hblk[b]));
    }
  }
  // With measured times, a block that could set the kernel's tail (more than twice the mean, and more than half the
  // time the kernel needs per workgroup slot: the total over about four resident workgroups per compute unit) is
  // dispatched in parts of SPLIT_TETS tets, each part its own workgroup with its own site box. Where items are short
  // against the kernel (large batches) nothing is split, since every part scans the sites again.
  if (learned && !(flags & RPD_NO_SPLIT) && !items.empty()) {
    unsigned long long sum = 0;
    for (unsigned long long c : cost) sum += c;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                hipSuccess || cus <= 0)
      cus = 256;
    const unsigned long long heavy = std::max(2 * (sum / items.size()), sum / (8ull * (unsigned long long)cus)) + 1;
    const size_t n0 = items.size();
    for (size_t q = 0; q < n0; ++q) {
      const int k = items[q].x, b = items[q].y;
      const int n = meshes[k]->hblk[b + 1] - meshes[k]->hblk[b];
      if (cost[q] < heavy || n <= SPLIT_TETS) continue;
      const int parts = (n + SPLIT_TETS - 1) / SPLIT_TETS;
      const unsigned long long c = cost[q] / parts + 1;
      items[q].y = b | (1 << ITEM_PART_SHIFT);
      cost[q] = c;
      for (int p = 2; p <= parts; ++p) {
        items.push_back(make_int2(k, b | (p << ITEM_PART_SHIFT)));
        cost.push_back(c);
      }
    }
  }
  // stable counting sort, descending, on the top bits of the cost range: about one bucket per item, 2^16 at most
  int bits = 8;
  while (bits < 16 && ((size_t)1 << bits) < items.size()) ++bits;
  const unsigned long long top = (1ull << bits) - 1;
  unsigned long long cmax = 1;
  for (unsigned long long c : cost) cmax = std::max(cmax, c);
  int shift = 0;
  while ((cmax >> shift) > top) ++shift;
  std::vector<int> start((size_t)top + 2, 0);
  for (unsigned long long c : cost) ++start[top - (c >> shift) + 1];
  for (size_t d = 0; d <= top; ++d) start[d + 1] += start[d];
  std::vector<int2> out(items.size());
  for (size_t k = 0; k < items.size(); ++k) out[start[top - (cost[k] >> shift)]++] = items[k];
  return out;
}

// Records the fast-kernel time of every item as its mesh's block costs (see work_items).
static void learn_costs(const std::vector<int2>& items, const unsigned* ticks,
                        const std::vector<ShapeDesc>& hd, const rpd_mesh* const* meshes) {
  const int nsh = (int)hd.size();
  std::vector<std::vector<unsigned>> per(nsh);
  for (int k = 0; k < nsh; ++k) per[k].assign(hd[k].nblk, 0);
  for (size_t k = 0; k < items.size(); ++k)  // a split block's cost is the sum of its parts'
    per[items[k].x][items[k].y & ((1 << ITEM_PART_SHIFT) - 1)] += ticks[k];
  for (int k = 0; k < nsh; ++k) {  // a mesh that several shapes share keeps the last one's times
    rpd_mesh* m = const_cast<rpd_mesh*>(meshes[k]);
    std::lock_guard<std::mutex> g(m->cost_mu);
    m->blk_cost.swap(per[k]);
  }
}

// What the site upload leaves in flight: kept by the caller until its stream has been synchronised.
struct SiteUpload {
  DBuf raw, dsrc;
  std::vector<SiteSrc> src;
};

// The site arrays of every shape as the validation kernel reads them: the caller's device arrays, or host arrays
// staged into one device buffer (copies queued on s).
static SiteUpload site_sources(const rpd_sites* sites, const std::vector<ShapeDesc>& hd, bool dev, hipStream_t s) {
  SiteUpload u;
  size_t total = 0;
  for (size_t k = 0; k < hd.size(); ++k) total += (size_t)sites[k].n_sites;
  DBuf& raw = u.raw;
  if (!dev) raw.alloc(sizeof(float) * 4 * total);
  std::vector<SiteSrc>& src = u.src;
  src.resize(hd.size());
  size_t pos = 0;
  for (size_t k = 0; k < hd.size(); ++k) {
    const rpd_sites* sp = &sites[k];
    const int n = sp->n_sites;
    SiteSrc& d = src[k];
    d.x = sp->sx;
    d.y = sp->sy;
    d.z = sp->sz;
    d.r = sp->sr;
    d.n = n;
    d.off = hd[k].site_off;
    if (!dev) {
      float* r = raw.as<float>() + pos;
      hip_check(hipMemcpyAsync(r, sp->sx, sizeof(float) * n, hipMemcpyHostToDevice, s), "upload");
      hip_check(hipMemcpyAsync(r + n, sp->sy, sizeof(float) * n, hipMemcpyHostToDevice, s), "upload");
      hip_check(hipMemcpyAsync(r + 2 * (size_t)n, sp->sz, sizeof(float) * n, hipMemcpyHostToDevice, s), "upload");
      hip_check(hipMemcpyAsync(r + 3 * (size_t)n, sp->sr, sizeof(float) * n, hipMemcpyHostToDevice, s), "upload");
      d.x = r;
      d.y = r + n;
      d.z = r + 2 * (size_t)n;
      d.r = r + 3 * (size_t)n;
      pos += 4 * (size_t)n;
    }
  }
  return u;
}

// the sites of every shape validated and packed into D.site by one launch
static SiteUpload upload_sites(DeviceState& D, const rpd_sites* sites, const std::vector<ShapeDesc>& hd, bool dev,
                               hipStream_t s) {
  SiteUpload u = site_sources(sites, hd, dev, s);
  const std::vector<SiteSrc>& src = u.src;
  int max_n = 0;
  for (const SiteSrc& d : src) max_n = std::max(max_n, d.n);
  u.dsrc.alloc(sizeof(SiteSrc) * std::max<size_t>(src.size(), 1));
  hip_check(hipMemcpyAsync(u.dsrc.p, src.data(), sizeof(SiteSrc) * src.size(), hipMemcpyHostToDevice, s), "upload");
  hip_check(launch_validate_sites_multi(u.dsrc.as<SiteSrc>(), (int)src.size(), max_n, D.site.as<float4>(),
                                        D.status.as<int>(), s),
            "validate sites");
  return u;
}

// All shapes of one call, one attempt. Returns false if a table ran out of room (caller retries larger).
static bool run_batch(const rpd_mesh* const* meshes, const rpd_sites* sites, int nsh, const rpd_opts& o,
                      hipStream_t s, int scale, std::vector<ShapeOut>& outs, rpd_stats& st) {
  const bool dev = (o.flags & RPD_DEVICE_PTRS) != 0;
  std::vector<int> nsites(nsh);
  for (int k = 0; k < nsh; ++k) nsites[k] = sites[k].n_sites;
  long long ns_tot = 0, nt_tot = 0;
  std::vector<ShapeDesc> hd = shape_table(meshes, nsites.data(), nsh, &ns_tot, &nt_tot);
  // the tables are cleared on the device while the host orders the work
  DeviceState D;
  D.alloc(nsh, (int)ns_tot, nt_tot, scale, (o.flags & RPD_KEEP_PIECES) != 0, false, fast_slots(o));
  D.clear(s);
  std::vector<int2> items = work_items(hd, meshes, o.flags);
  if (o.flags & RPD_SHUFFLE_QUEUE) {  // a fixed permutation: results must not depend on the processing order
    unsigned long long x = 0x9E3779B97F4A7C15ull;
    for (size_t k = items.size(); k > 1; --k) {
      x ^= x << 13;
      x ^= x >> 7;
      x ^= x << 17;
      std::swap(items[k - 1], items[x % k]);
    }
  }
  // the shape table, the site sources and the work items go up in one copy from pinned memory; then one launch
  // validates and packs every shape's sites (host site arrays are staged first)
  const size_t off_src = (sizeof(ShapeDesc) * nsh + 15) / 16 * 16;
  const size_t off_items = off_src + (sizeof(SiteSrc) * nsh + 15) / 16 * 16;
  const size_t stage_bytes = off_items + sizeof(int2) * std::max<size_t>(items.size(), 1);
  HostPinned stage(stage_bytes);  // released (back to the pool) after the stream is drained (below)
  DBuf dstage(stage_bytes);
  SiteUpload su = site_sources(sites, hd, dev, s);
  std::memcpy(stage.p, hd.data(), sizeof(ShapeDesc) * nsh);
  std::memcpy((unsigned char*)stage.p + off_src, su.src.data(), sizeof(SiteSrc) * nsh);
  if (!items.empty()) std::memcpy((unsigned char*)stage.p + off_items, items.data(), sizeof(int2) * items.size());
  hip_check(hipMemcpyAsync(dstage.p, stage.p, stage_bytes, hipMemcpyHostToDevice, s), "upload");
  const ShapeDesc* dshapes_p = (const ShapeDesc*)dstage.p;
  const int2* ditems_p = (const int2*)(dstage.as<unsigned char>() + off_items);
  int max_n = 0;
  for (int k = 0; k < nsh; ++k) max_n = std::max(max_n, sites[k].n_sites);
  hip_check(launch_validate_sites_multi((const SiteSrc*)(dstage.as<unsigned char>() + off_src), nsh, max_n,
                                        D.site.as<float4>(), D.status.as<int>(), s),
            "validate sites");
  const int kmax = o.clip_budget > 0 ? std::min(o.clip_budget, KMAX) : KMAX;
  ShapeArgs a = D.args(dshapes_p, ditems_p, (int)items.size(), o.flags, kmax);
  HostPinned ticks_host(sizeof(unsigned) * items.size() + 16);  // pinned: the copy does not stall the host
  struct DrainOnExit {  // an early exit (exception) must not leave the copy into ticks_host pending
    hipStream_t s;
    ~DrainOnExit() { (void)hipStreamSynchronize(s); }
  } drain{s};
  DBuf dcost(sizeof(unsigned) * std::max<size_t>(items.size(), 1));
  a.item_cost = dcost.as<unsigned>();
  Timing tm((o.flags & RPD_TIMING) != 0);
  tm.mark(0, s);
  hip_check(launch_clip_fast(a, o.precision, o.block, fast_slots(o), s), "clip kernel");
  tm.mark(1, s);
  if (!items.empty())  // read by the host after collect's synchronisation
    hip_check(hipMemcpyAsync(ticks_host.p, dcost.p, sizeof(unsigned) * items.size(), hipMemcpyDeviceToHost, s),
              "download");
  hip_check(launch_clip_slow(a, D.slow.as<unsigned char>(), D.waves, s), "deferred clip kernel");
  tm.mark(2, s);
  D.components(a, s);
  if (!collect(D, hd, dshapes_p, meshes, s, tm, outs, st)) return false;
  learn_costs(items, (const unsigned*)ticks_host.p, hd, meshes);
  st.n_items = (int64_t)items.size();
  st.ms_clip = tm.ms(0, 1);
  st.ms_deferred = tm.ms(1, 2);
  st.ms_reduce = tm.ms(2, 3);
  st.ms_total = tm.ms(0, 4);
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

const char* rpd_last_error(void) { return rpd::g_error; }

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
  info->owner_weights = m->owner;
  info->n_blocks = m->nblk;
  return RPD_OK;
}

void rpd_mesh_free(rpd_mesh* m) { delete m; }

static void check_opts(const rpd_opts& o) {
  if (o.precision != RPD_FP32_FALLBACK && o.precision != RPD_FP64) throw Failure{RPD_E_INVALID, "bad precision"};
  if (o.clip_budget != 0 && (o.clip_budget < 4 || o.clip_budget > rpd::KMAX))
    throw Failure{RPD_E_INVALID, "clip_budget must be 0 or in [4, 28]"};
  if (o.block != 0 && o.block != 64 && o.block != 128 && o.block != 256)
    throw Failure{RPD_E_INVALID, "block must be 0, 64, 128 or 256"};
  if (o.slots != 0 && o.slots != 12 && o.slots != 16) throw Failure{RPD_E_INVALID, "slots must be 0, 12 or 16"};
}

static void check_shapes(const rpd_mesh* const* meshes, const rpd_sites* sites, int32_t n_shapes) {
  if (!meshes || !sites || n_shapes <= 0) throw Failure{RPD_E_INVALID, "null argument or no shape"};
  if (n_shapes >= (1 << 16)) throw Failure{RPD_E_INVALID, "2^16 or more shapes in one call"};
  for (int k = 0; k < n_shapes; ++k) {
    const rpd_sites* sp = &sites[k];
    if (!meshes[k]) throw Failure{RPD_E_INVALID, "null mesh"};
    if (sp->n_sites <= 0 || sp->n_sites >= (1 << 21) || !sp->sx || !sp->sy || !sp->sz || !sp->sr)
      throw Failure{RPD_E_INVALID, "site count must be in [1, 2^21) with non-null arrays"};
  }
}

// Autotuner cache: launch shape (block, clip budget, vertex slots) of the FP32 path per (log2 mean sites per shape,
// log2 mean tets per shape) bucket, filled by rpd_autotune and read by rpd_build where block, clip_budget or slots
// is 0.
struct TuneShape {
  int block, budget, slots;
};
static std::mutex g_tune_mu;
static std::map<std::pair<int, int>, TuneShape> g_tune;


static std::pair<int, int> tune_bucket(const rpd_mesh* const* meshes, const rpd_sites* sites, int32_t n) {
  double ns = 0, nt = 0;
  for (int k = 0; k < n; ++k) {
    ns += sites[k].n_sites;
    nt += meshes[k]->nt;
  }
  return {(int)std::floor(std::log2(std::max(1.0, ns / n))), (int)std::floor(std::log2(std::max(1.0, nt / n)))};
}

static void apply_tuned(rpd_opts& o, const rpd_mesh* const* meshes, const rpd_sites* sites, int32_t n) {
  if (o.precision != RPD_FP32_FALLBACK || (o.block != 0 && o.clip_budget != 0 && o.slots != 0)) return;
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(tune_bucket(meshes, sites, n));
  if (it == g_tune.end()) return;
  if (o.block == 0) o.block = it->second.block;
  if (o.clip_budget == 0) o.clip_budget = it->second.budget;
  if (o.slots == 0) o.slots = it->second.slots;
}

static bool run_with_retry(const rpd_mesh* const* meshes, const rpd_sites* sites, int32_t n_shapes, const rpd_opts& o,
                           std::vector<rpd::ShapeOut>& shapes, rpd_stats& st) {
  hipStream_t s = (hipStream_t)o.stream;
  for (int scale = 1; scale <= 16; scale *= 2)
    if (rpd::run_batch(meshes, sites, n_shapes, o, s, scale, shapes, st)) return true;
  return false;
}

rpd_status rpd_build(const rpd_mesh* const* meshes, const rpd_sites* sites, int32_t n_shapes, const rpd_opts* opts,
                     rpd_result** out) {
  if (out) *out = nullptr;
  RPD_GUARD_BEGIN
  rpd::set_error("");
  if (!out) throw Failure{RPD_E_INVALID, "null argument"};
  rpd_opts o;
  std::memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  check_opts(o);
  check_shapes(meshes, sites, n_shapes);
  apply_tuned(o, meshes, sites, n_shapes);
  rpd_result* r = new rpd_result();
  std::memset(&r->stats, 0, sizeof(r->stats));
  try {
    r->shapes.resize(n_shapes);
    if (!run_with_retry(meshes, sites, n_shapes, o, r->shapes, r->stats))
      throw Failure{RPD_E_NOMEM, "result tables kept overflowing"};
  } catch (...) {
    delete r;
    throw;
  }
  *out = r;
  return RPD_OK;
  RPD_GUARD_END
}

rpd_status rpd_autotune(const rpd_mesh* const* meshes, const rpd_sites* sites, int32_t n_shapes, const rpd_opts* opts,
                        rpd_opts* best) {
  RPD_GUARD_BEGIN
  rpd::set_error("");
  if (!best) throw Failure{RPD_E_INVALID, "null argument"};
  rpd_opts o;
  std::memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  check_opts(o);
  check_shapes(meshes, sites, n_shapes);
  if (o.precision != RPD_FP32_FALLBACK) throw Failure{RPD_E_INVALID, "only the FP32 path is tuned"};
  o.flags |= RPD_TIMING;
  o.flags &= ~(uint32_t)RPD_KEEP_PIECES;
  // the default shape (64 threads, the full budget) is timed first; another shape replaces it only when it is
  // faster by more than 2%, so that shapes within the timing noise do not alternate from run to run
  const int cand[11][3] = {{64, rpd::KMAX, 16}, {64, 8, 16},  {64, 16, 16},  {128, 8, 16},         {128, 16, 16},
                           {128, rpd::KMAX, 16}, {256, 8, 16}, {256, 16, 16}, {256, rpd::KMAX, 16}, {64, rpd::KMAX, 12},
                           {64, 16, 12}};
  double best_ms = INFINITY;
  int bb = 64, bk = rpd::KMAX, bs = 16;
  for (const auto& sh : cand) {
    rpd_opts c = o;
    c.block = sh[0];
    c.clip_budget = sh[1];
    c.slots = sh[2];
    double ms = INFINITY;
    for (int rep = 0; rep < 3; ++rep) {  // the first run warms the allocator and the caches
      std::vector<rpd::ShapeOut> shapes(n_shapes);
      rpd_stats st;
      std::memset(&st, 0, sizeof(st));
      if (!run_with_retry(meshes, sites, n_shapes, c, shapes, st))
        throw Failure{RPD_E_NOMEM, "result tables kept overflowing"};
      if (rep > 0) ms = std::min(ms, st.ms_clip + st.ms_deferred);
    }
    if (ms < 0.98 * best_ms) {
      best_ms = ms;
      bb = sh[0];
      bk = sh[1];
      bs = sh[2];
    }
  }
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[tune_bucket(meshes, sites, n_shapes)] = {bb, bk, bs};
  }
  *best = opts ? *opts : o;
  best->block = bb;
  best->clip_budget = bk;
  best->slots = bs;
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

rpd_status rpd_edge_geometry(const rpd_result* r, int32_t shape, int64_t* n_out, const double** length,
                             const double** alpha) {
  rpd_status e = shape_check(r, shape);
  if (e) return e;
  if (!n_out) return RPD_E_INVALID;
  const rpd::ShapeOut& s = r->shapes[shape];
  *n_out = (int64_t)s.edge_len.size();
  if (length) *length = s.edge_len.data();
  if (alpha) *alpha = s.edge_alpha.data();
  return RPD_OK;
}

rpd_status rpd_medial_euler(const rpd_result* r, int32_t shape, int64_t* counts, int64_t* chi) {
  rpd_status e = shape_check(r, shape);
  if (e) return e;
  if (!counts) return RPD_E_INVALID;
  const rpd::ShapeOut& s = r->shapes[shape];
  counts[0] = (int64_t)std::count_if(s.cell_b0.begin(), s.cell_b0.end(), [](int32_t b) { return b > 0; });
  counts[1] = (int64_t)s.face_chi.size();
  counts[2] = (int64_t)s.edge_chi.size();
  counts[3] = (int64_t)s.rpv_keys.size() / 4;
  if (chi) *chi = counts[0] - counts[1] + counts[2] - counts[3];
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

rpd_status rpd_piece_terms(const rpd_result* r, int32_t shape, int32_t kind, int64_t* n_out, const int32_t** tet,
                           const int32_t** sites, const int64_t** num, const int32_t** glue) {
  rpd_status e = shape_check(r, shape);
  if (e) return e;
  if (!n_out || kind < RPD_CELL || kind > RPD_VERTEX) return RPD_E_INVALID;
  const rpd::ShapeOut& s = r->shapes[shape];
  const int q = kind - 1;
  *n_out = (int64_t)s.tm_t[q].size();
  if (tet) *tet = s.tm_t[q].data();
  if (sites) *sites = s.tm_s[q].data();
  if (num) *num = s.tm_num[q].data();
  if (glue) *glue = s.tm_glue[q].data();
  return RPD_OK;
}

void rpd_free(rpd_result* r) { delete r; }

}  // extern "C"

// ---------------------------------------------------------------------------------------------------------------
// incremental session
// ---------------------------------------------------------------------------------------------------------------
struct rpd_session {
  int device = 0;
  hipStream_t stream = nullptr;
  const rpd_mesh* mesh = nullptr;
  rpd_opts o{};
  int max_sites = 0, max_insert = 0, kmax = rpd::KMAX, mode = 0;
  bool failed = false;
  rpd::ShapeDesc hd{};
  rpd::DeviceState D;
  rpd::DBuf dshapes;  // [0] the shape before a round's insertions, [1] after them (the current state)
  rpd::DBuf all_items, items, table, tet_block, dirty, sel, selpos, best, ref, tet_used, ints;
  rpd::DBuf order;  // [nblk] blocks by their fast-kernel time in the initial build, heaviest first
  rpd::RoundState r{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int rounds = 0;
  double ms_last = 0;

  ~rpd_session() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

namespace rpd {

// int slots of rpd_session::ints
enum { SI_NSEL = 0, SI_NITEMS, SI_ROUND, SI_NS, SI_INS, SI_DIRTY, SI_COUNT };

static void check_status(rpd_session* S) {
  int hst = 0;
  hip_check(hipMemcpyAsync(&hst, S->D.status.p, sizeof(int), hipMemcpyDeviceToHost, S->stream), "download");
  hip_check(hipStreamSynchronize(S->stream), "synchronize");
  if (hst & ST_TABLE_FULL)
    throw Failure{RPD_E_NOMEM, "session tables are full: create the session with a larger max_sites"};
  status_error(hst);
}

// one full clipping pass over the items of a (all blocks, or the dirty ones with a device-side count)
static void clip_pass(rpd_session* S, const ShapeArgs& a) {
  hip_check(launch_fill_u64(S->D.cnt() + C_DEFER_ITEMS, 0, 1, S->stream), "fill");
  hip_check(launch_fill_u64(S->D.cnt() + C_DEFER2, 0, 1, S->stream), "fill");
  hip_check(launch_fill_u64(S->D.cnt() + C_LISTS, 0, 2, S->stream), "fill");  // C_LISTS and C_BIG
  hip_check(launch_clip_fast(a, S->o.precision, S->o.block, fast_slots(S->o), S->stream), "clip kernel");
  hip_check(launch_clip_slow(a, S->D.slow.as<unsigned char>(), S->D.waves, S->stream), "deferred clip kernel");
}

// Allocate at the given table scale, upload, compute the initial state. False if a table overflowed.
static bool session_init(rpd_session* S, const rpd_sites* sites, const rpd_sites* table, int scale) {
  const rpd_mesh* m = S->mesh;
  hipStream_t s = S->stream;
  const bool dev = (S->o.flags & RPD_DEVICE_PTRS) != 0;
  const int nt = m->nt, nblk = m->nblk;
  if (nblk >= (1 << ITEM_PART_SHIFT)) throw Failure{RPD_E_INVALID, "mesh with 2^20 or more workgroup blocks"};
  DeviceState& D = S->D;
  D.alloc(1, S->max_sites, nt, scale, false, true, fast_slots(S->o));
  D.clear(s);
  std::vector<ShapeDesc> hd{S->hd};
  const SiteUpload su = upload_sites(D, sites, hd, dev, s);
  struct DrainOnExit {  // the upload's buffers are released only after the stream has drained
    hipStream_t s;
    ~DrainOnExit() { (void)hipStreamSynchronize(s); }
  } drain{s};
  const size_t nslots = S->mode ? 4 * (size_t)nt : (size_t)nt;
  S->tet_used.alloc(sizeof(int) * nslots);
  hip_check(launch_fill_i32(S->tet_used.as<int>(), S->mode ? 1 : 0, nslots, s), "fill");
  if (S->mode) {  // shrunk spheres at every surface face (the pins), on the grid
    DBuf tri(36 * 4 * (size_t)nt), pin(12 * 4 * (size_t)nt), nrm(12 * 4 * (size_t)nt), slot(16 * (size_t)nt),
        own(16 * (size_t)nt), cnt(sizeof(int)), sph;
    hip_check(launch_fill_i32(cnt.as<int>(), 0, 1, s), "fill");
    hip_check(launch_surface_faces(m->tp.as<float4>(), m->tn.as<int>(), nt, tri.as<float>(), pin.as<float>(),
                                   nrm.as<float>(), slot.as<int>(), cnt.as<int>(), s),
              "surface faces");
    int nf = 0;
    hip_check(hipMemcpyAsync(&nf, cnt.p, sizeof(int), hipMemcpyDeviceToHost, s), "download");
    hip_check(hipStreamSynchronize(s), "synchronize");
    sph.alloc(16 * (size_t)std::max(nf, 1));
    hip_check(launch_iota(own.as<int>(), nf, s), "iota");
    shrink_spheres(tri.as<float>(), nf, pin.as<float>(), nrm.as<float>(), own.as<int>(), nf, s, sph.as<float4>());
    S->table.alloc(sizeof(float4) * nslots);
    hip_check(launch_scatter_spheres(sph.as<float4>(), slot.as<int>(), nf, S->table.as<float4>(),
                                     S->tet_used.as<int>(), s),
              "table");
    hip_check(hipStreamSynchronize(s), "synchronize");
  } else {  // the table, validated like sites, kept in the caller's tet order (the pick rule's numbering)
    DBuf stage;
    const float *tx = table->sx, *ty = table->sy, *tz = table->sz, *tr = table->sr;
    if (!dev) {
      stage.alloc(sizeof(float) * 4 * (size_t)nt);
      float* q = stage.as<float>();
      hip_check(hipMemcpyAsync(q, tx, sizeof(float) * nt, hipMemcpyHostToDevice, s), "upload");
      hip_check(hipMemcpyAsync(q + nt, ty, sizeof(float) * nt, hipMemcpyHostToDevice, s), "upload");
      hip_check(hipMemcpyAsync(q + 2 * (size_t)nt, tz, sizeof(float) * nt, hipMemcpyHostToDevice, s), "upload");
      hip_check(hipMemcpyAsync(q + 3 * (size_t)nt, tr, sizeof(float) * nt, hipMemcpyHostToDevice, s), "upload");
      tx = q;
      ty = q + nt;
      tz = q + 2 * (size_t)nt;
      tr = q + 3 * (size_t)nt;
    }
    S->table.alloc(sizeof(float4) * (size_t)nt);
    hip_check(launch_validate_sites(tx, ty, tz, tr, nt, S->table.as<float4>(), D.status.as<int>(), s),
              "validate table");
    hip_check(hipStreamSynchronize(s), "synchronize");  // the staging buffers are released next
  }
  std::vector<int> tb(nt);
  for (int b = 0; b < nblk; ++b)
    for (int t = m->hblk[b]; t < m->hblk[b + 1]; ++t) tb[t] = b;
  std::vector<int2> all(nblk);
  for (int b = 0; b < nblk; ++b) all[b] = make_int2(0, b);
  ShapeDesc two[2] = {S->hd, S->hd};
  two[0].sign = -1;  // the state before a round's insertions: its dirty pieces are taken back
  S->dshapes.alloc(sizeof(two));
  S->all_items.alloc(sizeof(int2) * (size_t)nblk);
  S->items.alloc(sizeof(int2) * 2 * (size_t)nblk * (TB / SPLIT_TETS));  // every dirty block in parts, twice
  S->tet_block.alloc(sizeof(int) * (size_t)nt);
  S->dirty.alloc(sizeof(unsigned long long) * (size_t)nblk);
  S->sel.alloc(sizeof(int) * (size_t)S->max_insert);
  S->best.alloc(8 * (size_t)S->max_insert);
  S->ref.alloc(sizeof(unsigned long long) * (size_t)S->max_insert);
  S->selpos.alloc(sizeof(int) * (size_t)S->max_sites);
  S->ints.alloc(sizeof(int) * SI_COUNT);
  hip_check(hipMemcpyAsync(S->dshapes.p, two, sizeof(two), hipMemcpyHostToDevice, s), "upload");
  hip_check(hipMemcpyAsync(S->all_items.p, all.data(), sizeof(int2) * all.size(), hipMemcpyHostToDevice, s),
            "upload");
  hip_check(hipMemcpyAsync(S->tet_block.p, tb.data(), sizeof(int) * tb.size(), hipMemcpyHostToDevice, s), "upload");
  hip_check(launch_fill_i32(S->dirty.as<int>(), 0, 2 * (size_t)nblk, s), "fill");
  hip_check(launch_fill_i32(S->selpos.as<int>(), -1, S->max_sites, s), "fill");
  hip_check(launch_fill_i32(S->ints.as<int>(), 0, SI_COUNT, s), "fill");
  hip_check(launch_fill_i32(S->ints.as<int>() + SI_NS, S->hd.ns, 1, s), "fill");

  ShapeDesc* ds = S->dshapes.as<ShapeDesc>();
  ShapeArgs a = D.args(ds + 1, S->all_items.as<int2>(), nblk, S->o.flags, S->kmax);
  DBuf ticks(sizeof(unsigned) * (size_t)nblk);
  a.item_cost = ticks.as<unsigned>();  // item k is block k
  clip_pass(S, a);
  D.components(a, s);
  hip_check(hipStreamSynchronize(s), "synchronize");
  int hst = 0;
  hip_check(hipMemcpy(&hst, D.status.p, sizeof(int), hipMemcpyDeviceToHost), "download");
  if (hst & ST_TABLE_FULL) return false;
  status_error(hst);
  {  // the rounds scan the blocks heaviest first (k_dirty_items)
    std::vector<unsigned> cost(nblk);
    hip_check(hipMemcpy(cost.data(), ticks.p, sizeof(unsigned) * (size_t)nblk, hipMemcpyDeviceToHost), "download");
    std::vector<int> ord(nblk);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    S->order.alloc(sizeof(int) * (size_t)nblk);
    hip_check(hipMemcpy(S->order.p, ord.data(), sizeof(int) * (size_t)nblk, hipMemcpyHostToDevice), "upload");
  }

  int* ints = S->ints.as<int>();
  RoundState& r = S->r;
  r.nsel = ints + SI_NSEL;
  r.sel = S->sel.as<int>();
  r.selpos = S->selpos.as<int>();
  r.best = S->best.as<unsigned long long>();
  r.ref = S->ref.as<unsigned long long>();
  r.perm = m->perm.as<int>();
  r.tet_used = S->tet_used.as<int>();
  r.table = S->table.as<float4>();
  r.mode = S->mode;
  r.tet_block = S->tet_block.as<int>();
  r.dirty = S->dirty.as<unsigned long long>();
  r.order = S->order.as<int>();
  r.items = S->items.as<int2>();
  r.blk = m->blk.as<int>();
  r.clist = D.clist.as<int>();
  r.cseg = D.cseg.as<int>();
  r.clen = glue_segment_length((size_t)D.capN);
  r.cnseg = (int)((size_t)D.capN / r.clen);
  r.nitems = ints + SI_NITEMS;
  r.round = ints + SI_ROUND;
  r.ns_cur = ints + SI_NS;
  r.ins_total = ints + SI_INS;
  r.dirty_total = ints + SI_DIRTY;
  r.old_desc = ds;
  r.new_desc = ds + 1;
  r.max_sites = S->max_sites;
  r.max_insert = S->max_insert;
  return true;
}

// the launch sequence of one round (captured once into the session's graph)
static void session_round(rpd_session* S) {
  hipStream_t s = S->stream;
  DeviceState& D = S->D;
  const rpd_mesh* m = S->mesh;
  ShapeDesc* ds = S->dshapes.as<ShapeDesc>();
  // one launch takes out the dirty parts' pieces of the state before the round's insertions (shape 0, sign -1)
  // and adds those of the state after them (shape 1): items come in pairs (0, part), (1, part)
  ShapeArgs a = D.args(ds, S->items.as<int2>(), m->nblk, S->o.flags, S->kmax);
  ShapeArgs a_new = D.args(ds + 1, S->items.as<int2>(), m->nblk, S->o.flags, S->kmax);
  a.nitems_dev = S->r.nitems;
  // the dirty items are counted on the device: a grid of twice the resident workgroups (five per compute unit)
  // takes them in grid-stride order, instead of one workgroup per possible item that mostly exit at once
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device) != hipSuccess || cus <= 0) cus = 256;
  a.nitems = std::min(2 * m->nblk * (TB / SPLIT_TETS), 10 * cus);
  D.set_touch(a);
  D.set_touch(a_new);
  hip_check(launch_round_front(S->r, a_new, D.cell_b0.as<int>(), m->tp.as<float4>(), m->nt,
                               m->nblk, s),
            "round selection");
  clip_pass(S, a);
  hip_check(launch_touch_removed(a_new, s), "changed pieces");
  D.components(a_new, s);
  hip_check(launch_round_end(S->r, s), "round end");
}

static void session_capture(rpd_session* S) {
  hip_check(hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal), "begin capture");
  try {
    session_round(S);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(S->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hip_check(hipStreamEndCapture(S->stream, &S->graph), "end capture");
  hip_check(hipGraphInstantiate(&S->exec, S->graph, nullptr, nullptr, 0), "graph instantiate");
}

struct DeviceGuard {  // make the session's device current for the call, restore the caller's afterwards
  int prev = -1;
  explicit DeviceGuard(int dev) {
    hip_check(hipGetDevice(&prev), "hipGetDevice");
    if (prev != dev) hip_check(hipSetDevice(dev), "hipSetDevice");
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace rpd

extern "C" {

rpd_status rpd_session_create(const rpd_mesh* mesh, const rpd_sites* sites, const rpd_sites* table,
                              const rpd_session_opts* opts, rpd_session** out) {
  if (out) *out = nullptr;
  RPD_GUARD_BEGIN
  rpd::set_error("");
  if (!mesh || !sites || !opts || !out) throw Failure{RPD_E_INVALID, "null argument"};
  if (opts->insertion != RPD_INSERT_TABLE && opts->insertion != RPD_INSERT_SHRINK)
    throw Failure{RPD_E_INVALID, "unknown insertion mode"};
  if (opts->insertion == RPD_INSERT_TABLE && !table) throw Failure{RPD_E_INVALID, "null table"};
  rpd_opts o = opts->build;
  check_opts(o);
  {  // the autotuner's launch shape
    const rpd_mesh* ms1[1] = {mesh};
    apply_tuned(o, ms1, sites, 1);
  }
  if (o.flags & (RPD_KEEP_PIECES | RPD_FORCE_SLOW_PATH))
    throw Failure{RPD_E_INVALID, "RPD_KEEP_PIECES and RPD_FORCE_SLOW_PATH are not available in a session"};
  if (sites->n_sites <= 0 || !sites->sx || !sites->sy || !sites->sz || !sites->sr)
    throw Failure{RPD_E_INVALID, "no initial sites"};
  if (opts->max_sites < sites->n_sites || opts->max_sites >= (1 << 21))
    throw Failure{RPD_E_INVALID, "max_sites must be in [n_sites, 2^21)"};
  if (opts->max_insert < 1 || opts->max_insert > rpd::MAX_INSERT)
    throw Failure{RPD_E_INVALID, "max_insert must be in [1, 4096]"};
  if (opts->insertion == RPD_INSERT_TABLE &&
      (table->n_sites != mesh->nt || !table->sx || !table->sy || !table->sz || !table->sr))
    throw Failure{RPD_E_INVALID, "the table needs one sphere per tet"};
  if (mesh->nblk <= 0) throw Failure{RPD_E_INVALID, "empty mesh"};
  // the session reads the inputs on a non-blocking stream of its own, which is not ordered after the caller's
  // stream: wait for that stream (NULL: the null stream) before anything is read
  rpd::hip_check(hipStreamSynchronize((hipStream_t)o.stream), "synchronize");
  rpd_session* S = new rpd_session();
  try {
    rpd::hip_check(hipGetDevice(&S->device), "hipGetDevice");
    if (S->device != mesh->device) throw Failure{RPD_E_INVALID, "the mesh lives on another device"};
    S->mesh = mesh;
    S->o = o;
    S->max_sites = opts->max_sites;
    S->max_insert = opts->max_insert;
    S->mode = opts->insertion;
    S->kmax = o.clip_budget > 0 ? std::min(o.clip_budget, rpd::KMAX) : rpd::KMAX;
    rpd::hip_check(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking), "stream");
    for (auto& e : S->ev) rpd::hip_check(hipEventCreate(&e), "hipEventCreate");
    int n0 = sites->n_sites;
    long long ns_tot = 0, nt_tot = 0;
    const rpd_mesh* ms[1] = {mesh};
    S->hd = rpd::shape_table(ms, &n0, 1, &ns_tot, &nt_tot)[0];
    bool done = false;
    for (int scale = 2; scale <= 16 && !done; scale *= 2) done = rpd::session_init(S, sites, table, scale);
    if (!done) throw Failure{RPD_E_NOMEM, "session tables kept overflowing"};
    rpd::session_capture(S);
  } catch (...) {
    delete S;
    throw;
  }
  *out = S;
  return RPD_OK;
  RPD_GUARD_END
}

rpd_status rpd_session_run(rpd_session* S, int32_t rounds) {
  RPD_GUARD_BEGIN
  rpd::set_error("");
  if (!S || rounds < 0) throw Failure{RPD_E_INVALID, "null session or negative round count"};
  if (S->failed) throw Failure{RPD_E_INVALID, "the session failed earlier"};
  rpd::DeviceGuard g(S->device);
  try {
    rpd::hip_check(hipEventRecord(S->ev[0], S->stream), "hipEventRecord");
    for (int k = 0; k < rounds; ++k) rpd::hip_check(hipGraphLaunch(S->exec, S->stream), "graph launch");
    rpd::hip_check(hipEventRecord(S->ev[1], S->stream), "hipEventRecord");
    rpd::check_status(S);
    float ms = 0;
    rpd::hip_check(hipEventElapsedTime(&ms, S->ev[0], S->ev[1]), "hipEventElapsedTime");
    S->ms_last = ms;
    S->rounds += rounds;
  } catch (...) {
    S->failed = true;
    throw;
  }
  return RPD_OK;
  RPD_GUARD_END
}

rpd_status rpd_session_get_info(rpd_session* S, rpd_session_info* info) {
  RPD_GUARD_BEGIN
  if (!S || !info) throw Failure{RPD_E_INVALID, "null argument"};
  rpd::DeviceGuard g(S->device);
  int h[rpd::SI_COUNT];
  rpd::hip_check(hipMemcpyAsync(h, S->ints.p, sizeof(h), hipMemcpyDeviceToHost, S->stream), "download");
  rpd::hip_check(hipStreamSynchronize(S->stream), "synchronize");
  info->n_sites = h[rpd::SI_NS];
  info->rounds = S->rounds;
  info->n_selected = h[rpd::SI_NSEL];
  info->n_blocks = S->mesh->nblk;
  info->n_inserted = h[rpd::SI_INS];
  info->n_dirty_blocks = h[rpd::SI_DIRTY];
  unsigned long long tot[rpd::NCOUNTERS + 8];
  S->D.totals(tot, S->stream);
  info->n_clipped = (int64_t)tot[rpd::C_CAND];
  info->ms_last_run = S->ms_last;
  return RPD_OK;
  RPD_GUARD_END
}

rpd_status rpd_session_sites(rpd_session* S, int32_t cap, float* xyzr, int32_t* n_out) {
  RPD_GUARD_BEGIN
  if (!S || !xyzr || !n_out) throw Failure{RPD_E_INVALID, "null argument"};
  rpd::DeviceGuard g(S->device);
  int n = 0;
  rpd::hip_check(hipMemcpyAsync(&n, S->ints.as<int>() + rpd::SI_NS, sizeof(int), hipMemcpyDeviceToHost, S->stream),
                 "download");
  rpd::hip_check(hipStreamSynchronize(S->stream), "synchronize");
  if (n > cap) throw Failure{RPD_E_INVALID, "output buffer too small for the session's sites"};
  rpd::hip_check(hipMemcpyAsync(xyzr, S->D.site.p, sizeof(float4) * (size_t)n, hipMemcpyDeviceToHost, S->stream),
                 "download");
  rpd::hip_check(hipStreamSynchronize(S->stream), "synchronize");
  *n_out = n;
  return RPD_OK;
  RPD_GUARD_END
}

rpd_status rpd_session_result(rpd_session* S, rpd_result** out) {
  if (out) *out = nullptr;
  RPD_GUARD_BEGIN
  rpd::set_error("");
  if (!S || !out) throw Failure{RPD_E_INVALID, "null argument"};
  if (S->failed) throw Failure{RPD_E_INVALID, "the session failed earlier"};
  rpd::DeviceGuard g(S->device);
  int n = 0;
  rpd::hip_check(hipMemcpyAsync(&n, S->ints.as<int>() + rpd::SI_NS, sizeof(int), hipMemcpyDeviceToHost, S->stream),
                 "download");
  rpd::hip_check(hipStreamSynchronize(S->stream), "synchronize");
  std::vector<rpd::ShapeDesc> hd{S->hd};
  hd[0].ns = n;
  rpd_result* r = new rpd_result();
  std::memset(&r->stats, 0, sizeof(r->stats));
  try {
    r->shapes.resize(1);
    rpd::Timing tm(false);
    const rpd_mesh* ms[1] = {S->mesh};
    if (!rpd::collect(S->D, hd, S->dshapes.as<rpd::ShapeDesc>() + 1, ms, S->stream, tm, r->shapes, r->stats))
      throw Failure{RPD_E_NOMEM, "session tables are full"};
  } catch (...) {
    delete r;
    throw;
  }
  *out = r;
  return RPD_OK;
  RPD_GUARD_END
}

void rpd_session_free(rpd_session* S) {
  if (!S) return;
  const int dev = S->device;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != dev) (void)hipSetDevice(dev);
  delete S;
  if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
}

}  // extern "C"
