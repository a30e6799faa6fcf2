// Medial spheres by sphere shrinking (Sec. 5.1, Fig. tech_sphere_gen (a)): the maximal ball that is tangent to the
// surface at a pin point p (inward unit normal n) and contains no surface point in its interior.
//
// The shrinking iteration replaces the radius by the radius of the ball through p and the surface point nearest to
// the current centre until the ball is empty; its fixed point is known in closed form. A surface point q lies strictly
// inside the ball of centre p + r n and radius r iff r > rho(q) = |q - p|^2 / (2 n.(q - p)) (for n.(q - p) > 0), so the
// maximal empty ball has radius r* = min over surface points q of rho(q). Over one triangle the smallest rho is
// reached where the growing ball first touches it: at a vertex, at a stationary point of rho along an edge (a
// quadratic in the edge parameter), or at the point where the ball is tangent to the triangle's plane (if that point
// lies in the triangle). The kernel takes that minimum over every surface triangle (brute force, the same traversal
// as the geometric-error metric), so no iteration and no nearest-point search is needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "rpd.h"
#include "rpd_host.h"
#include "rpd_launch.h"

namespace rpd {
namespace {

constexpr int SHR_THREADS = 256;
constexpr int SHR_R = 2;  // pins per thread

// rho at q = p + w (w = q - p): |w|^2 / (2 n.w) where n.w > 0, else +inf
__device__ inline float rho_of(float wx, float wy, float wz, float nx, float ny, float nz) {
  const float l = nx * wx + ny * wy + nz * wz;
  return l > 0.f ? (wx * wx + wy * wy + wz * wz) / (2.f * l) : INFINITY;
}

// smallest rho along the edge a + s e, s in (0, 1): stationary points of |w + s e|^2 / (2 (alpha + beta s)),
// roots of A beta s^2 + 2 A alpha s + (2 B alpha - C beta) = 0 with A = e.e, B = w.e, C = w.w
__device__ inline float edge_rho(float wx, float wy, float wz, float ex, float ey, float ez, float nx, float ny,
                                 float nz) {
  const float A = ex * ex + ey * ey + ez * ez, B = wx * ex + wy * ey + wz * ez, C = wx * wx + wy * wy + wz * wz;
  const float al = nx * wx + ny * wy + nz * wz, be = nx * ex + ny * ey + nz * ez;
  float best = INFINITY;
  auto take = [&](float s) {
    if (s > 0.f && s < 1.f) {
      const float L = al + be * s;
      if (L > 0.f) best = fminf(best, (C + s * (2.f * B + s * A)) / (2.f * L));
    }
  };
  const float qa = A * be, qb = 2.f * A * al, qc = 2.f * B * al - C * be;
  if (fabsf(qa) > 1e-30f) {
    const float disc = qb * qb - 4.f * qa * qc;
    if (disc >= 0.f) {
      const float sd = __builtin_amdgcn_sqrtf(disc);
      take((-qb + sd) / (2.f * qa));
      take((-qb - sd) / (2.f * qa));
    }
  } else if (fabsf(qb) > 1e-30f) {
    take(-qc / qb);
  }
  return best;
}

// triangle records: (a, 0) (e1 = b - a, 0) (e2 = c - a, 0) (unit normal m, 0) (dual basis u1 of e1, e2) (u2), as six
// float4, in FP64 then rounded; u1.e1 = 1, u1.e2 = 0 and u2 the other way round give barycentric coordinates
__global__ void k_shrink_prep(const float* tri, long long nt, float4* rec) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < nt; t += (long long)gridDim.x * blockDim.x) {
    const float* v = tri + 9 * t;
    const double ax = v[0], ay = v[1], az = v[2];
    const double e1x = v[3] - ax, e1y = v[4] - ay, e1z = v[5] - az;
    const double e2x = v[6] - ax, e2y = v[7] - ay, e2z = v[8] - az;
    double mx = e1y * e2z - e1z * e2y, my = e1z * e2x - e1x * e2z, mz = e1x * e2y - e1y * e2x;
    const double mm = sqrt(mx * mx + my * my + mz * mz);
    const double g11 = e1x * e1x + e1y * e1y + e1z * e1z, g12 = e1x * e2x + e1y * e2y + e1z * e2z,
                 g22 = e2x * e2x + e2y * e2y + e2z * e2z;
    const double det = g11 * g22 - g12 * g12;
    float4* R = rec + 6 * t;
    R[0] = make_float4(v[0], v[1], v[2], 0.f);
    R[1] = make_float4((float)e1x, (float)e1y, (float)e1z, 0.f);
    R[2] = make_float4((float)e2x, (float)e2y, (float)e2z, 0.f);
    if (mm > 0.0 && det > 0.0) {
      mx /= mm;
      my /= mm;
      mz /= mm;
      const double i11 = g22 / det, i12 = -g12 / det, i22 = g11 / det;
      R[3] = make_float4((float)mx, (float)my, (float)mz, 1.f);
      R[4] = make_float4((float)(i11 * e1x + i12 * e2x), (float)(i11 * e1y + i12 * e2y), (float)(i11 * e1z + i12 * e2z),
                         0.f);
      R[5] = make_float4((float)(i12 * e1x + i22 * e2x), (float)(i12 * e1y + i22 * e2y), (float)(i12 * e1z + i22 * e2z),
                         0.f);
    } else {  // degenerate triangle: vertices and edges only
      R[3] = make_float4(0.f, 0.f, 0.f, 0.f);
      R[4] = make_float4(0.f, 0.f, 0.f, 0.f);
      R[5] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

__global__ __launch_bounds__(SHR_THREADS) void k_shrink(const float4* __restrict__ rec, long long nt,
                                                        const float* __restrict__ pin, const float* __restrict__ nrm,
                                                        const int* __restrict__ own, long long n,
                                                        unsigned* __restrict__ best_bits) {
  const int chunks = gridDim.y, c = blockIdx.y;
  const long long base = (long long)blockIdx.x * (SHR_THREADS * SHR_R) + threadIdx.x;
  float px[SHR_R], py[SHR_R], pz[SHR_R], nx[SHR_R], ny[SHR_R], nz[SHR_R], best[SHR_R];
  long long skip[SHR_R];
  for (int r = 0; r < SHR_R; ++r) {
    const long long s = base + (long long)r * SHR_THREADS;
    const long long sc = s < n ? s : n - 1;
    px[r] = pin[3 * sc];
    py[r] = pin[3 * sc + 1];
    pz[r] = pin[3 * sc + 2];
    nx[r] = nrm[3 * sc];
    ny[r] = nrm[3 * sc + 1];
    nz[r] = nrm[3 * sc + 2];
    skip[r] = own ? own[sc] : -1;
    best[r] = INFINITY;
  }
  const long long t0 = nt * c / chunks, t1 = nt * (c + 1) / chunks;
  for (long long t = t0; t < t1; ++t) {
    const float4* R = rec + 6 * t;
    const float4 A = R[0], E1 = R[1], E2 = R[2], M = R[3], U1 = R[4], U2 = R[5];
    for (int r = 0; r < SHR_R; ++r) {
      // vertices
      const float wx = A.x - px[r], wy = A.y - py[r], wz = A.z - pz[r];
      float v = rho_of(wx, wy, wz, nx[r], ny[r], nz[r]);
      v = fminf(v, rho_of(wx + E1.x, wy + E1.y, wz + E1.z, nx[r], ny[r], nz[r]));
      v = fminf(v, rho_of(wx + E2.x, wy + E2.y, wz + E2.z, nx[r], ny[r], nz[r]));
      // edges a->b, a->c, b->c
      v = fminf(v, edge_rho(wx, wy, wz, E1.x, E1.y, E1.z, nx[r], ny[r], nz[r]));
      v = fminf(v, edge_rho(wx, wy, wz, E2.x, E2.y, E2.z, nx[r], ny[r], nz[r]));
      v = fminf(v, edge_rho(wx + E1.x, wy + E1.y, wz + E1.z, E2.x - E1.x, E2.y - E1.y, E2.z - E1.z, nx[r], ny[r],
                            nz[r]));
      // tangency to the plane m.x = m.a at a point of the triangle: |m.(p + r n) - m.a| = r
      if (M.w != 0.f) {
        const float dl = -(M.x * wx + M.y * wy + M.z * wz);  // m.(p - a)
        const float mu = M.x * nx[r] + M.y * ny[r] + M.z * nz[r];
        for (int sg = 0; sg < 2; ++sg) {
          const float den = sg ? -(1.f + mu) : (1.f - mu);
          const float rr = dl / den;
          if (den != 0.f && rr > 0.f) {
            // tangent point relative to a: p + rr n - (m.(p + rr n - a)) m - a
            const float h = dl + rr * mu;
            const float tx = -wx + rr * nx[r] - h * M.x, ty = -wy + rr * ny[r] - h * M.y, tz = -wz + rr * nz[r] - h * M.z;
            const float b1 = U1.x * tx + U1.y * ty + U1.z * tz, b2 = U2.x * tx + U2.y * ty + U2.z * tz;
            if (b1 >= 0.f && b2 >= 0.f && b1 + b2 <= 1.f) v = fminf(v, rr);
          }
        }
      }
      if (t != skip[r]) best[r] = fminf(best[r], v);
    }
  }
  for (int r = 0; r < SHR_R; ++r) {
    const long long s = base + (long long)r * SHR_THREADS;
    if (s < n && best[r] < INFINITY) atomicMin(&best_bits[s], __float_as_uint(best[r]));  // positive floats
  }
}

__global__ void k_shrink_finish(const unsigned* bits, const float* pin, const float* nrm, long long n, float4* out) {
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < n; s += (long long)gridDim.x * blockDim.x) {
    const float r = bits[s] == 0xffffffffu ? INFINITY : __uint_as_float(bits[s]);
    out[s] = make_float4(pin[3 * s] + r * nrm[3 * s], pin[3 * s + 1] + r * nrm[3 * s + 1],
                         pin[3 * s + 2] + r * nrm[3 * s + 2], r);
  }
}

}  // namespace

void shrink_spheres(const float* tri, long long nt, const float* pins, const float* normals, const int* own,
                    long long n, hipStream_t st, float4* out) {
  DBuf rec(16 * 6 * (size_t)std::max<long long>(nt, 1)), bits(4 * (size_t)std::max<long long>(n, 1));
  if (n == 0) return;
  hip_check(launch_fill_i32(bits.as<int>(), -1, (size_t)n, st), "fill");
  if (nt > 0) {
    hipLaunchKernelGGL(k_shrink_prep, dim3((unsigned)std::min<long long>((nt + 255) / 256, 4096)), dim3(256), 0, st,
                       tri, nt, rec.as<float4>());
    const long long blocks = (n + SHR_THREADS * SHR_R - 1) / (SHR_THREADS * SHR_R);
    long long chunks = std::max<long long>(1, std::min<long long>((2048 + blocks - 1) / blocks, nt / 32));
    chunks = std::min<long long>(chunks, 65535);
    hipLaunchKernelGGL(k_shrink, dim3((unsigned)blocks, (unsigned)chunks), dim3(SHR_THREADS), 0, st, rec.as<float4>(),
                       nt, pins, normals, own, n, bits.as<unsigned>());
    hip_check(hipGetLastError(), "shrink");
  }
  hipLaunchKernelGGL(k_shrink_finish, dim3((unsigned)std::min<long long>((n + 255) / 256, 4096)), dim3(256), 0, st,
                     bits.as<unsigned>(), pins, normals, n, out);
  hip_check(hipGetLastError(), "shrink finish");
}

}  // namespace rpd

extern "C" rpd_status rpd_shrink_spheres(const float* tris, int64_t n_tris, const float* pins, const float* normals,
                                         const int32_t* own_tri, int64_t n_pins, uint32_t flags, void* stream,
                                         float* spheres) {
  try {
    rpd::set_error("");
    if (n_tris < 0 || n_pins < 0) throw rpd::Failure{RPD_E_INVALID, "negative count"};
    if ((n_tris && !tris) || (n_pins && (!pins || !normals || !spheres)))
      throw rpd::Failure{RPD_E_INVALID, "null array"};
    if (n_pins == 0) return RPD_OK;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) throw rpd::Failure{RPD_E_DEVICE, "no HIP device"};
    hipStream_t st = (hipStream_t)stream;
    const bool dev = (flags & RPD_DEVICE_PTRS) != 0;
    if (dev) {
      rpd::shrink_spheres(tris, n_tris, pins, normals, own_tri, n_pins, st, (float4*)spheres);
    } else {
      rpd::DBuf t(36 * (size_t)n_tris), p(12 * (size_t)n_pins), q(12 * (size_t)n_pins), o(4 * (size_t)n_pins),
          out(16 * (size_t)n_pins);
      if (n_tris) rpd::hip_check(hipMemcpyAsync(t.p, tris, 36 * (size_t)n_tris, hipMemcpyHostToDevice, st), "upload");
      rpd::hip_check(hipMemcpyAsync(p.p, pins, 12 * (size_t)n_pins, hipMemcpyHostToDevice, st), "upload");
      rpd::hip_check(hipMemcpyAsync(q.p, normals, 12 * (size_t)n_pins, hipMemcpyHostToDevice, st), "upload");
      if (own_tri)
        rpd::hip_check(hipMemcpyAsync(o.p, own_tri, 4 * (size_t)n_pins, hipMemcpyHostToDevice, st), "upload");
      rpd::shrink_spheres(t.as<float>(), n_tris, p.as<float>(), q.as<float>(), own_tri ? o.as<int>() : nullptr, n_pins,
                          st, out.as<float4>());
      rpd::hip_check(hipMemcpyAsync(spheres, out.p, 16 * (size_t)n_pins, hipMemcpyDeviceToHost, st), "download");
    }
    rpd::hip_check(hipStreamSynchronize(st), "synchronize");
    return RPD_OK;
  } catch (const rpd::Failure& f) {
    rpd::set_error(f.msg);
    return f.code;
  } catch (const std::bad_alloc&) {
    rpd::set_error("host allocation failed");
    return RPD_E_NOMEM;
  }
}
