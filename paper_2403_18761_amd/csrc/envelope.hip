// Distance from surface samples to the enveloping volume of a medial mesh (Sec. 4.3, geometric preservation).
//
// The enveloping volume of a medial vertex is its sphere, of an edge the medial cone (spheres interpolated linearly
// between its two end spheres) and of a triangle the medial slab (spheres interpolated over the triangle), Sec. 3.2.
// For a sample q and an element whose spheres are B(c(t), r(t)), t over a segment or a triangle, the value is
// min_t |q - c(t)| - r(t): the Euclidean distance to the element's volume when q is outside it, minus the depth
// when inside. The result per sample is the minimum over every element of the mesh, and the element reaching it.
//
// The function of t is convex, so its minimum over an element lies either at an interior stationary point or on the
// element's boundary, and the boundary of a cone (its end spheres) and of a slab (its three cones) are elements of
// the mesh themselves when the mesh lists every face of its simplices. Each element is therefore evaluated only at
// its interior stationary point, in closed form (k = slope of r along a unit cone axis, g = in-plane gradient of r
// over a slab, d = q - c_1):
//   sphere: |d| - r
//   cone:   h sqrt(1 - k^2) - k u - r_1, with u = d . axis, h = |d x axis|, valid when the stationary axial position
//           u + k h / sqrt(1 - k^2) lies in [0, L]  (|k| < 1; otherwise one end sphere contains the other)
//   slab:   |H| sqrt(1 - |g|^2) - g . d - r_1, with H = d . normal, valid when the stationary centre
//           q - H normal + g |H| / sqrt(1 - |g|^2) lies in the triangle  (|g| < 1)
// and an element whose stationary point falls outside is left to its boundary elements.
//
// Brute force over all elements (the work the paper puts on the GPU): each thread keeps four samples in registers,
// element records are read with uniform (scalar) loads, and the element lists are split into chunks over the grid's
// second dimension so that the launch fills the chip; per-sample minima meet in one 64-bit atomicMin of
// (order-preserving float bits, element id), which also breaks exact ties towards the lower element id.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "rpd.h"
#include "rpd_host.h"
#include "rpd_launch.h"

namespace rpd {
namespace {

constexpr int ENV_THREADS = 256;
constexpr int ENV_R = 4;  // samples per thread
constexpr int ENV_SAMPLES_PER_BLOCK = ENV_THREADS * ENV_R;
constexpr int CONE_F4 = 3, SLAB_F4 = 5;

__device__ inline double3 sub3(double3 a, double3 b) { return make_double3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline double dot3(double3 a, double3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline double3 cross3(double3 a, double3 b) {
  return make_double3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ inline double3 c3(float4 s) { return make_double3(s.x, s.y, s.z); }
__device__ inline float4 f4(double3 v, double w) { return make_float4((float)v.x, (float)v.y, (float)v.z, (float)w); }

// element records, in FP64 then rounded: cone = (c1, r1) (axis, L) (k, sqrt(1-k^2), k / sqrt(1-k^2), 0);
// slab = (c1, r1) (normal, sqrt(1-|g|^2)) (g, s m1.g) (m1, s m2.g) (m2, 0) with s = 1 / sqrt(1 - |g|^2) and
// (m1, m2) the in-plane dual basis of the triangle's edge vectors e1 = c2 - c1, e2 = c3 - c1
__global__ void k_env_prep(const float4* sph, int ns, const int* edges, int ne, const int* tris, int nf,
                           float4* cone, float4* slab, int* status) {
  const int n = ne + nf;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    if (q < ne) {
      const int i = edges[2 * q], j = edges[2 * q + 1];
      float4* R = cone + CONE_F4 * (size_t)q;
      if (i < 0 || j < 0 || i >= ns || j >= ns) {
        atomicOr(status, ST_INVALID);
        R[0] = make_float4(0.f, 0.f, 0.f, 0.f);
        R[1] = make_float4(0.f, 0.f, 0.f, -1.f);
        R[2] = make_float4(0.f, 0.f, 0.f, 0.f);
        continue;
      }
      const float4 a = sph[i], b = sph[j];
      const double3 e = sub3(c3(b), c3(a));
      const double L = sqrt(dot3(e, e)), dr = (double)b.w - (double)a.w;
      R[0] = a;
      if (L > 0.0 && fabs(dr) < L) {
        const double k = dr / L, sq = sqrt(1.0 - k * k);
        R[1] = f4(make_double3(e.x / L, e.y / L, e.z / L), L);
        R[2] = make_float4((float)k, (float)sq, (float)(k / sq), 0.f);
      } else {  // one end sphere contains the other: no interior stationary point
        R[1] = make_float4(0.f, 0.f, 0.f, -1.f);
        R[2] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    } else {
      const int f = q - ne;
      const int i = tris[3 * f], j = tris[3 * f + 1], k = tris[3 * f + 2];
      float4* R = slab + SLAB_F4 * (size_t)f;
      const float4 inert[SLAB_F4] = {make_float4(0.f, 0.f, 0.f, -INFINITY), make_float4(0.f, 0.f, 0.f, 0.f),
                                     make_float4(0.f, 0.f, 0.f, 0.f), make_float4(0.f, 0.f, 0.f, 0.f),
                                     make_float4(0.f, 0.f, 0.f, 0.f)};  // value +inf everywhere
      if (i < 0 || j < 0 || k < 0 || i >= ns || j >= ns || k >= ns) {
        atomicOr(status, ST_INVALID);
        for (int w = 0; w < SLAB_F4; ++w) R[w] = inert[w];
        continue;
      }
      const float4 a = sph[i], b = sph[j], c = sph[k];
      const double3 e1 = sub3(c3(b), c3(a)), e2 = sub3(c3(c), c3(a));
      const double g11 = dot3(e1, e1), g12 = dot3(e1, e2), g22 = dot3(e2, e2);
      const double det = g11 * g22 - g12 * g12;
      bool ok = det > 1e-12 * g11 * g22;  // sin^2 of the corner angle; thinner slabs are left to their cones
      double3 m1 = make_double3(0, 0, 0), m2 = m1, g = m1, nrm = m1;
      double gg = 1.0;
      if (ok) {
        const double i11 = g22 / det, i12 = -g12 / det, i22 = g11 / det;
        m1 = make_double3(i11 * e1.x + i12 * e2.x, i11 * e1.y + i12 * e2.y, i11 * e1.z + i12 * e2.z);
        m2 = make_double3(i12 * e1.x + i22 * e2.x, i12 * e1.y + i22 * e2.y, i12 * e1.z + i22 * e2.z);
        const double d1 = (double)b.w - (double)a.w, d2 = (double)c.w - (double)a.w;
        g = make_double3(d1 * m1.x + d2 * m2.x, d1 * m1.y + d2 * m2.y, d1 * m1.z + d2 * m2.z);
        gg = dot3(g, g);
        const double3 nc = cross3(e1, e2);
        const double nn = sqrt(dot3(nc, nc));
        nrm = make_double3(nc.x / nn, nc.y / nn, nc.z / nn);
        ok = gg < 1.0;
      }
      if (!ok) {  // degenerate triangle, or one sphere's cone contains the slab's interior: boundary only
        for (int w = 0; w < SLAB_F4; ++w) R[w] = inert[w];
        continue;
      }
      const double sq = sqrt(1.0 - gg), s = 1.0 / sq;
      R[0] = a;
      R[1] = f4(nrm, sq);
      R[2] = f4(g, s * dot3(m1, g));
      R[3] = f4(m1, s * dot3(m2, g));
      R[4] = f4(m2, 0.0);
    }
  }
}

// float -> unsigned with the same order (negative values included)
__device__ inline unsigned order_bits(float f) {
  const unsigned b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float from_order_bits(unsigned k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// running minimum of a sample; with ID the element reaching it too (strict: the lower id of a chunk keeps a tie)
template <bool ID>
__device__ inline void keep_min(float f, int id, float& best, int& best_id) {
  if (ID) {
    if (f < best) {
      best = f;
      best_id = id;
    }
  } else {
    best = fminf(best, f);
  }
}

template <bool ID>
__global__ __launch_bounds__(ENV_THREADS) void k_env_dist(const float* __restrict__ xyz, long long n,
                                                          const float4* __restrict__ sph, int ns,
                                                          const float4* __restrict__ cone, int ne,
                                                          const float4* __restrict__ slab, int nf,
                                                          unsigned long long* __restrict__ best_key) {
  const int chunks = gridDim.y, c = blockIdx.y;
  const long long base = (long long)blockIdx.x * ENV_SAMPLES_PER_BLOCK + threadIdx.x;
  float qx[ENV_R], qy[ENV_R], qz[ENV_R], best[ENV_R];
  int bid[ENV_R];
  for (int r = 0; r < ENV_R; ++r) {
    const long long s = base + (long long)r * ENV_THREADS;
    const long long sc = s < n ? s : (n - 1);
    qx[r] = xyz[3 * sc];
    qy[r] = xyz[3 * sc + 1];
    qz[r] = xyz[3 * sc + 2];
    best[r] = INFINITY;
    bid[r] = ID ? -1 : 0;
  }
  // this chunk's share of each list (uniform bounds)
  const int s0 = (int)((long long)ns * c / chunks), s1 = (int)((long long)ns * (c + 1) / chunks);
  const int e0 = (int)((long long)ne * c / chunks), e1 = (int)((long long)ne * (c + 1) / chunks);
  const int f0 = (int)((long long)nf * c / chunks), f1 = (int)((long long)nf * (c + 1) / chunks);

  for (int p = s0; p < s1; ++p) {
    const float4 S = sph[p];
    for (int r = 0; r < ENV_R; ++r) {
      const float dx = qx[r] - S.x, dy = qy[r] - S.y, dz = qz[r] - S.z;
      keep_min<ID>(__builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz) - S.w, p, best[r], bid[r]);
    }
  }
  for (int p = e0; p < e1; ++p) {
    const float4 A = cone[CONE_F4 * (size_t)p], B = cone[CONE_F4 * (size_t)p + 1], K = cone[CONE_F4 * (size_t)p + 2];
    for (int r = 0; r < ENV_R; ++r) {
      const float dx = qx[r] - A.x, dy = qy[r] - A.y, dz = qz[r] - A.z;
      const float u = dx * B.x + dy * B.y + dz * B.z;
      const float cx = dy * B.z - dz * B.y, cy = dz * B.x - dx * B.z, cz = dx * B.y - dy * B.x;
      const float h = __builtin_amdgcn_sqrtf(cx * cx + cy * cy + cz * cz);
      const float t = u + K.z * h;
      const float f = (t >= 0.f && t <= B.w) ? K.y * h - K.x * u - A.w : INFINITY;
      keep_min<ID>(f, ns + p, best[r], bid[r]);
    }
  }
  for (int p = f0; p < f1; ++p) {
    const float4* R = slab + SLAB_F4 * (size_t)p;
    const float4 A = R[0], Nn = R[1], G = R[2], M1 = R[3], M2 = R[4];
    for (int r = 0; r < ENV_R; ++r) {
      const float dx = qx[r] - A.x, dy = qy[r] - A.y, dz = qz[r] - A.z;
      const float aH = fabsf(dx * Nn.x + dy * Nn.y + dz * Nn.z);
      const float gd = dx * G.x + dy * G.y + dz * G.z;
      const float al = dx * M1.x + dy * M1.y + dz * M1.z + aH * G.w;
      const float be = dx * M2.x + dy * M2.y + dz * M2.z + aH * M1.w;
      const bool in = al >= 0.f && be >= 0.f && al + be <= 1.f;
      keep_min<ID>(in ? aH * Nn.w - gd - A.w : INFINITY, ns + ne + p, best[r], bid[r]);
    }
  }
  for (int r = 0; r < ENV_R; ++r) {
    const long long s = base + (long long)r * ENV_THREADS;
    if (s < n && (ID ? bid[r] >= 0 : best[r] < INFINITY))
      atomicMin(&best_key[s], ((unsigned long long)order_bits(best[r]) << 32) | (unsigned)bid[r]);
  }
}

__global__ void k_env_finish(const unsigned long long* key, long long n, float* dist, int* nearest) {
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < n; s += (long long)gridDim.x * blockDim.x) {
    const unsigned long long k = key[s];
    const bool none = k == ~0ull;
    dist[s] = none ? INFINITY : from_order_bits((unsigned)(k >> 32));
    if (nearest) nearest[s] = none ? -1 : (int)(k & 0xffffffffu);
  }
}

// Working memory of one call: the element records (CONE_F4 float4 per edge, SLAB_F4 per triangle), the per-sample
// minima (one 64-bit key per sample) and a status word.
size_t record_bytes(long long ne, long long nf) { return 16 * ((size_t)CONE_F4 * ne + (size_t)SLAB_F4 * nf); }

// The launches of one call on device-resident inputs and outputs, given its working memory; ev0/ev1 (optional)
// bracket the distance kernel. No allocation and no exception: returns the first HIP error.
hipError_t envelope_launch(const float4* sph, int ns, const int* edg, long long ne, const int* tri, long long nf,
                           const float* xyz, long long n, hipStream_t st, float4* rec, unsigned long long* key,
                           int* status, float* dist, int* nearest, hipEvent_t ev0, hipEvent_t ev1) {
  float4* cone = rec;
  float4* slab = rec + (size_t)CONE_F4 * ne;
  hipError_t e = launch_fill_i32(status, 0, 1, st);
  if (e == hipSuccess) e = launch_fill_u64(key, ~0ull, (size_t)n, st);
  if (e != hipSuccess) return e;
  if (ne + nf > 0) {
    const int g = (int)std::min<long long>((ne + nf + 255) / 256, 4096);
    hipLaunchKernelGGL(k_env_prep, dim3(g), dim3(256), 0, st, sph, ns, edg, (int)ne, tri, (int)nf, cone, slab,
                       status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // grid: sample blocks x element chunks, about 2048 workgroups in all, each chunk at least 64 elements
  const long long sblocks = (n + ENV_SAMPLES_PER_BLOCK - 1) / ENV_SAMPLES_PER_BLOCK;
  const long long total = ns + ne + nf;
  long long chunks = std::max<long long>(1, std::min<long long>((2048 + sblocks - 1) / sblocks, total / 64));
  chunks = std::min<long long>(chunks, 65535);
  if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
  if (total > 0) {
    if (nearest)
      hipLaunchKernelGGL(k_env_dist<true>, dim3((unsigned)sblocks, (unsigned)chunks), dim3(ENV_THREADS), 0, st, xyz,
                         n, sph, ns, cone, (int)ne, slab, (int)nf, key);
    else
      hipLaunchKernelGGL(k_env_dist<false>, dim3((unsigned)sblocks, (unsigned)chunks), dim3(ENV_THREADS), 0, st, xyz,
                         n, sph, ns, cone, (int)ne, slab, (int)nf, key);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (ev1 && (e = hipEventRecord(ev1, st)) != hipSuccess) return e;
  const int g = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_env_finish, dim3(g), dim3(256), 0, st, key, n, dist, nearest);
  return hipGetLastError();
}

// argument checks shared by both entry points (pure: no device access); 0 when the call may proceed
rpd_status envelope_args(const float* spheres, int ns, const int* edges, long long ne, const int* tris, long long nf,
                         const float* samples, long long n, const float* dist, const char** msg) {
  *msg = "";
  if (ns < 0 || ne < 0 || nf < 0 || n < 0) return *msg = "negative count", RPD_E_INVALID;
  if (ns + ne + nf > (long long)INT32_MAX) return *msg = "more than 2^31 elements", RPD_E_INVALID;
  if ((ns && !spheres) || (ne && !edges) || (nf && !tris) || (n && (!samples || !dist)))
    return *msg = "null array", RPD_E_INVALID;
  if ((n + ENV_SAMPLES_PER_BLOCK - 1) / ENV_SAMPLES_PER_BLOCK > INT32_MAX) return *msg = "too many samples", RPD_E_INVALID;
  return RPD_OK;
}

void envelope_distance(const float* spheres, int ns, const int* edges, long long ne, const int* tris, long long nf,
                       const float* samples, long long n, unsigned flags, hipStream_t st, float* dist, int* nearest,
                       float* kernel_ms) {
  const char* msg = "";
  if (rpd_status c = envelope_args(spheres, ns, edges, ne, tris, nf, samples, n, dist, &msg)) throw Failure{c, msg};
  if (n == 0) return;
  const bool dev = (flags & RPD_DEVICE_PTRS) != 0;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) throw Failure{RPD_E_DEVICE, "no HIP device"};

  DBuf d_sph, d_edge, d_tri, d_xyz, d_out, d_near;
  const float4* sph = (const float4*)spheres;
  const int* edg = edges;
  const int* tri = tris;
  const float* xyz = samples;
  if (!dev) {  // stage host inputs
    d_sph.alloc(16 * (size_t)ns);
    d_edge.alloc(8 * (size_t)ne);
    d_tri.alloc(12 * (size_t)nf);
    d_xyz.alloc(12 * (size_t)n);
    if (ns) hip_check(hipMemcpyAsync(d_sph.p, spheres, 16 * (size_t)ns, hipMemcpyHostToDevice, st), "upload");
    if (ne) hip_check(hipMemcpyAsync(d_edge.p, edges, 8 * (size_t)ne, hipMemcpyHostToDevice, st), "upload");
    if (nf) hip_check(hipMemcpyAsync(d_tri.p, tris, 12 * (size_t)nf, hipMemcpyHostToDevice, st), "upload");
    hip_check(hipMemcpyAsync(d_xyz.p, samples, 12 * (size_t)n, hipMemcpyHostToDevice, st), "upload");
    sph = d_sph.as<float4>();
    edg = d_edge.as<int>();
    tri = d_tri.as<int>();
    xyz = d_xyz.as<float>();
  }
  DBuf rec(record_bytes(ne, nf)), key(8 * (size_t)n), status(sizeof(int));
  hipEvent_t ev[2] = {nullptr, nullptr};
  struct EventGuard {
    hipEvent_t* e;
    ~EventGuard() {
      for (int k = 0; k < 2; ++k)
        if (e[k]) (void)hipEventDestroy(e[k]);
    }
  } ev_guard{ev};
  if (kernel_ms) {
    *kernel_ms = 0.f;
    for (auto& e : ev) hip_check(hipEventCreate(&e), "hipEventCreate");
  }
  float* out_d = dist;
  int* out_n = nearest;
  if (!dev) {
    d_out.alloc(4 * (size_t)n);
    if (nearest) d_near.alloc(4 * (size_t)n);
    out_d = d_out.as<float>();
    out_n = nearest ? d_near.as<int>() : nullptr;
  }
  hip_check(envelope_launch(sph, ns, edg, ne, tri, nf, xyz, n, st, rec.as<float4>(), key.as<unsigned long long>(),
                            status.as<int>(), out_d, out_n, ev[0], ev[1]),
            "envelope distance");
  int hst = 0;
  hip_check(hipMemcpyAsync(&hst, status.p, sizeof(int), hipMemcpyDeviceToHost, st), "download");
  if (!dev) {
    hip_check(hipMemcpyAsync(dist, out_d, 4 * (size_t)n, hipMemcpyDeviceToHost, st), "download");
    if (nearest) hip_check(hipMemcpyAsync(nearest, out_n, 4 * (size_t)n, hipMemcpyDeviceToHost, st), "download");
  }
  hip_check(hipStreamSynchronize(st), "synchronize");
  if (kernel_ms) hip_check(hipEventElapsedTime(kernel_ms, ev[0], ev[1]), "hipEventElapsedTime");
  if (hst & ST_INVALID) throw Failure{RPD_E_INVALID, "an edge or triangle names a sphere out of range"};
}

// ---------------------------------------------------------------------------------------------------------------
// The no-allocation variant's working memory: one fixed region per device, reserved with the library's code
// object and held until the process ends. Host code never passes the array itself to a kernel (its name is a host
// stand-in); it looks up the region's device address once per device and uses that.
// ---------------------------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[RPD_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES];  // device address of `scratch` per device (nullptr until looked up)

// the current device's address of the region (looked up on the first call on that device)
rpd_status scratch_address(void** out, const char** msg) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return *msg = "no HIP device", RPD_E_DEVICE;
  if (dev >= MAX_DEVICES) return *msg = "device index beyond the scratch table", RPD_E_DEVICE;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return *msg = "scratch region not available on this device", RPD_E_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RPD_OK;
}

// bytes of the region one call uses: status word, per-sample minima, element records, each 256-byte aligned
size_t noalloc_bytes(long long ne, long long nf, long long n) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return 256 + up(8 * (size_t)n) + up(record_bytes(ne, nf));
}
}  // namespace
}  // namespace rpd

extern "C" rpd_status rpd_envelope_distance_noalloc(const float* spheres, int32_t n_spheres, const int32_t* edges,
                                                    int64_t n_edges, const int32_t* tris, int64_t n_tris,
                                                    const float* samples, int64_t n_samples, void* stream, float* dist,
                                                    int32_t* nearest) {
  using namespace rpd;
  const char* msg = "";
  rpd_status c = envelope_args(spheres, n_spheres, edges, n_edges, tris, n_tris, samples, n_samples, dist, &msg);
  if (c == RPD_OK && noalloc_bytes(n_edges, n_tris, n_samples) > (size_t)RPD_NOALLOC_SCRATCH_BYTES) {
    c = RPD_E_NOMEM;
    msg = "the samples and elements exceed the no-allocation scratch region (RPD_NOALLOC_SCRATCH_BYTES)";
  }
  if (c != RPD_OK) {
    set_error(msg);
    return c;
  }
  set_error("");
  if (n_samples == 0) return RPD_OK;
  void* base = nullptr;
  if ((c = scratch_address(&base, &msg)) != RPD_OK) {
    set_error(msg);
    return c;
  }
  unsigned char* b = (unsigned char*)base;
  int* status = (int*)b;
  unsigned long long* key = (unsigned long long*)(b + 256);
  float4* rec = (float4*)(b + 256 + ((8 * (size_t)n_samples + 255) & ~(size_t)255));
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = envelope_launch((const float4*)spheres, n_spheres, edges, n_edges, tris, n_tris, samples, n_samples,
                                 st, rec, key, status, dist, nearest, nullptr, nullptr);
  int hst = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hst, status, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    set_error(hipGetErrorString(e));
    return RPD_E_DEVICE;
  }
  if (hst & ST_INVALID) {
    set_error("an edge or triangle names a sphere out of range");
    return RPD_E_INVALID;
  }
  return RPD_OK;
}

extern "C" rpd_status rpd_envelope_distance(const float* spheres, int32_t n_spheres, const int32_t* edges,
                                            int64_t n_edges, const int32_t* tris, int64_t n_tris,
                                            const float* samples, int64_t n_samples, uint32_t flags, void* stream,
                                            float* dist, int32_t* nearest, float* kernel_ms) {
  try {
    rpd::set_error("");
    rpd::envelope_distance(spheres, n_spheres, edges, n_edges, tris, n_tris, samples, n_samples, flags,
                           (hipStream_t)stream, dist, nearest, kernel_ms);
    return RPD_OK;
  } catch (const rpd::Failure& f) {
    rpd::set_error(f.msg);
    return f.code;
  } catch (const std::bad_alloc&) {
    rpd::set_error("host allocation failed");
    return RPD_E_NOMEM;
  }
}
