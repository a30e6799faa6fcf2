// Device-side building blocks of the restricted-power-diagram clipping (paper Sec. 5.2 Tet-Cell clipping with the
// half-space polytope representation of Sec. 5.2 -- planes + vertices as plane triples -- and the fractional Euler
// characteristic of Sec. 4.1.2). Everything here is written for gfx950 wave64; the plane constructions and the FP64
// filter are also compiled for the host, where a test checks them against exact arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rpd.h"
#include "rpd_common.h"

namespace rpd {

// predicate helpers that the host test build also compiles
#define RPD_HD __host__ __device__

// ---------------------------------------------------------------------------------------------------------------
// precision traits
// ---------------------------------------------------------------------------------------------------------------
template <typename T>
struct Prec;
template <>
struct Prec<float> {
  static constexpr float u = 5.9604644775390625e-08f;  // 2^-24, unit roundoff
  static constexpr float tiny = 1e-30f;                 // absolute floor covering underflow
};
template <>
struct Prec<double> {
  static constexpr double u = 1.1102230246251565e-16;  // 2^-53
  static constexpr double tiny = 1e-290;
};

template <typename T>
struct Plane {
  T nx, ny, nz, d;  // kept side: n.x + d >= 0, x in the tet-local frame (origin = tet vertex 0)
};

__device__ inline float pow2_scale(float m) {
  int e;
  frexpf(m, &e);
  return ldexpf(1.0f, -e);
}
__device__ inline double pow2_scale(double m) {
  int e;
  frexp(m, &e);
  return ldexp(1.0, -e);
}

// Scale by a power of two (exact) so that max |n| lies in [1/2, 1).
template <typename T>
__device__ inline Plane<T> normalise(Plane<T> p) {
  T m = fmax(fabs(p.nx), fmax(fabs(p.ny), fabs(p.nz)));
  T s = pow2_scale(m);
  p.nx *= s;
  p.ny *= s;
  p.nz *= s;
  p.d *= s;
  return p;
}

// ---------------------------------------------------------------------------------------------------------------
// Vertex construction: the meet of three normalised planes as Cartesian coordinates plus F, a bound such that for
// any normalised plane q the rounding error of q(x~) against the exact q(x*) is at most F + 4.001 u |d_q|.
// Derivation (inputs carry relative error <= u, max |n| <= 1):
//   X = -(d_a n_b x n_c + d_b n_c x n_a + d_c n_a x n_b), W = n_a . (n_b x n_c); at most 8 roundings per monomial
//   (3 input + 5 arithmetic) => |X~ - X| <= g8 * 2 (|d_a|+|d_b|+|d_c|), |W~ - W| <= 6 g8, g8 = 8u/(1-8u);
//   x = X/W with one division and one product (<= 4u relative); when |W~| >= 12 g8,
//   E = 2 [g8 (2 D3 + 6 |x~|) / |W~| + 4u |x~|] bounds |x~ - x*| componentwise;
//   the plane evaluation by three fused multiply-adds adds (g3 + u)(3|x~| + |d|) and the vertex error 3E.
// ---------------------------------------------------------------------------------------------------------------
template <typename T>
__device__ inline void make_vertex(const Plane<T>& A, const Plane<T>& B, const Plane<T>& C, T& x, T& y, T& z, T& F) {
  const T u = Prec<T>::u;
  T bcx = fma(B.ny, C.nz, -(B.nz * C.ny)), bcy = fma(B.nz, C.nx, -(B.nx * C.nz)), bcz = fma(B.nx, C.ny, -(B.ny * C.nx));
  T cax = fma(C.ny, A.nz, -(C.nz * A.ny)), cay = fma(C.nz, A.nx, -(C.nx * A.nz)), caz = fma(C.nx, A.ny, -(C.ny * A.nx));
  T abx = fma(A.ny, B.nz, -(A.nz * B.ny)), aby = fma(A.nz, B.nx, -(A.nx * B.nz)), abz = fma(A.nx, B.ny, -(A.ny * B.nx));
  T W = fma(A.nx, bcx, fma(A.ny, bcy, A.nz * bcz));
  T X = -fma(A.d, bcx, fma(B.d, cax, C.d * abx));
  T Y = -fma(A.d, bcy, fma(B.d, cay, C.d * aby));
  T Z = -fma(A.d, bcz, fma(B.d, caz, C.d * abz));
  T aW = fabs(W);
  const T g8 = T(8.001) * u;
  if (!(aW >= T(12) * g8)) {  // ill-conditioned (or NaN): every predicate on this vertex is escalated
    x = y = z = T(0);
    F = T(INFINITY);
    return;
  }
  T inv = T(1) / W;
  x = X * inv;
  y = Y * inv;
  z = Z * inv;
  T xm = fmax(fabs(x), fmax(fabs(y), fabs(z)));
  T D3 = fabs(A.d) + fabs(B.d) + fabs(C.d);
  T E = T(2.0001) * (g8 * (T(2) * D3 + T(6) * xm) / aW + T(4) * u * xm);
  F = (T(12.001) * u * xm + T(3.001) * E) * (T(1) + T(1.0 / 1048576.0)) + Prec<T>::tiny;
}

// bound term of an exactly known point (a tet vertex): only the evaluation rounding
template <typename T>
__device__ inline T exact_point_F(T x, T y, T z) {
  T xm = fmax(fabs(x), fmax(fabs(y), fabs(z)));
  return T(12.001) * Prec<T>::u * xm * (T(1) + T(1.0 / 1048576.0)) + Prec<T>::tiny;
}

// +1 / -1 when certain, 0 when |value| is within the bound.
template <typename T>
__device__ inline int side_fast(const Plane<T>& q, T x, T y, T z, T F) {
  T s = fma(q.nz, z, fma(q.ny, y, fma(q.nx, x, q.d)));
  T B = F + T(4.001 * (1.0 + 1.0 / 1048576.0)) * Prec<T>::u * fabs(q.d);
  if (s > B) return 1;
  if (s < -B) return -1;
  return 0;
}

// FP64 homogeneous test with a semi-static bound: sign of plane q at the meet of planes a, b, c, computed as
// sign(n_q . X + d_q W) * sign(W) from exactly representable (or once-rounded) coefficients. Returns 0 if uncertain.
RPD_HD inline int side64(const Plane<double>& A, const Plane<double>& B, const Plane<double>& C,
                             const Plane<double>& Q) {
  const double u = Prec<double>::u;
  double bcx = fma(B.ny, C.nz, -(B.nz * C.ny)), bcy = fma(B.nz, C.nx, -(B.nx * C.nz)),
         bcz = fma(B.nx, C.ny, -(B.ny * C.nx));
  double cax = fma(C.ny, A.nz, -(C.nz * A.ny)), cay = fma(C.nz, A.nx, -(C.nx * A.nz)),
         caz = fma(C.nx, A.ny, -(C.ny * A.nx));
  double abx = fma(A.ny, B.nz, -(A.nz * B.ny)), aby = fma(A.nz, B.nx, -(A.nx * B.nz)),
         abz = fma(A.nx, B.ny, -(A.ny * B.nx));
  double W = fma(A.nx, bcx, fma(A.ny, bcy, A.nz * bcz));
  double X = -fma(A.d, bcx, fma(B.d, cax, C.d * abx));
  double Y = -fma(A.d, bcy, fma(B.d, cay, C.d * aby));
  double Z = -fma(A.d, bcz, fma(B.d, caz, C.d * abz));
  double s = fma(Q.nx, X, fma(Q.ny, Y, fma(Q.nz, Z, Q.d * W)));
  // magnitudes: the same expressions on absolute values
  double bax = fabs(B.ny) * fabs(C.nz) + fabs(B.nz) * fabs(C.ny);
  double bay = fabs(B.nz) * fabs(C.nx) + fabs(B.nx) * fabs(C.nz);
  double baz = fabs(B.nx) * fabs(C.ny) + fabs(B.ny) * fabs(C.nx);
  double cax_ = fabs(C.ny) * fabs(A.nz) + fabs(C.nz) * fabs(A.ny);
  double cay_ = fabs(C.nz) * fabs(A.nx) + fabs(C.nx) * fabs(A.nz);
  double caz_ = fabs(C.nx) * fabs(A.ny) + fabs(C.ny) * fabs(A.nx);
  double abx_ = fabs(A.ny) * fabs(B.nz) + fabs(A.nz) * fabs(B.ny);
  double aby_ = fabs(A.nz) * fabs(B.nx) + fabs(A.nx) * fabs(B.nz);
  double abz_ = fabs(A.nx) * fabs(B.ny) + fabs(A.ny) * fabs(B.nx);
  double Wa = fabs(A.nx) * bax + fabs(A.ny) * bay + fabs(A.nz) * baz;
  double Xa = fabs(A.d) * bax + fabs(B.d) * cax_ + fabs(C.d) * abx_;
  double Ya = fabs(A.d) * bay + fabs(B.d) * cay_ + fabs(C.d) * aby_;
  double Za = fabs(A.d) * baz + fabs(B.d) * caz_ + fabs(C.d) * abz_;
  double sa = fabs(Q.nx) * Xa + fabs(Q.ny) * Ya + fabs(Q.nz) * Za + fabs(Q.d) * Wa;
  // W: <= 5 roundings; s: <= 9 roundings + 1 input rounding of a face offset; margins 8u and 12u
  if (!(fabs(W) > 8.0 * u * Wa + Prec<double>::tiny)) return 0;
  if (!(fabs(s) > 12.0 * u * sa + Prec<double>::tiny)) return 0;
  return ((s > 0) == (W > 0)) ? 1 : -1;
}

// ---------------------------------------------------------------------------------------------------------------
// Exact integer predicate (grid units 2^-20, tet-local origin). 256-bit two's complement arithmetic.
// ---------------------------------------------------------------------------------------------------------------
typedef unsigned long long u64;
typedef __int128 i128;
typedef unsigned __int128 u128;

struct I256 {
  u64 w[4];
};

__device__ inline I256 i256(i128 v) {
  I256 r;
  r.w[0] = (u64)v;
  r.w[1] = (u64)((u128)v >> 64);
  u64 s = v < 0 ? ~0ull : 0ull;
  r.w[2] = s;
  r.w[3] = s;
  return r;
}
__device__ inline I256 i256_add(const I256& a, const I256& b) {
  I256 r;
  u128 c = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c += (u128)a.w[k] + b.w[k];
    r.w[k] = (u64)c;
    c >>= 64;
  }
  return r;
}
__device__ inline I256 i256_neg(const I256& a) {
  I256 r;
  u128 c = 1;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c += (u128)(~a.w[k]);
    r.w[k] = (u64)c;
    c >>= 64;
  }
  return r;
}
__device__ inline bool i256_isneg(const I256& a) { return (a.w[3] >> 63) != 0; }
__device__ inline I256 i256_mul(I256 a, I256 b) {
  bool na = i256_isneg(a), nb = i256_isneg(b);
  if (na) a = i256_neg(a);
  if (nb) b = i256_neg(b);
  I256 r = {{0, 0, 0, 0}};
  for (int i = 0; i < 4; ++i) {
    u128 carry = 0;
    for (int j = 0; i + j < 4; ++j) {
      u128 t = (u128)a.w[i] * b.w[j] + r.w[i + j] + carry;
      r.w[i + j] = (u64)t;
      carry = t >> 64;
    }
  }
  return (na != nb) ? i256_neg(r) : r;
}
__device__ inline int i256_sign(const I256& a) {
  if (i256_isneg(a)) return -1;
  return (a.w[0] | a.w[1] | a.w[2] | a.w[3]) ? 1 : 0;
}

struct PlaneI {
  long long nx, ny, nz;  // |n| < 2^45
  i128 d;                // |d| < 2^69
};

// Exact sign of plane Q at the meet of A, B, C; returns 2 if A, B, C do not meet in one point.
//
// An exact zero is resolved by symbolic perturbation of the weights (simulation of simplicity): site s gets
// r_s^2 + eps_s with eps_s infinitesimal and eps_0 >> eps_1 >> ... (a lower site id dominates). A bisector of the
// cell's site i against site j (offset D_j - D_i, D = power distance of the local origin) then has offset
// d + eps_i - eps_j, face planes are unchanged, and the raw value below, linear in the four offsets, gains
// sum_P c_P (eps_i - eps_j(P)) with c_P the cofactor of plane P's offset. Its sign is that of the lowest site's
// nonzero coefficient; Q's own site has coefficient -W != 0, so the result is never 0. site[] holds the other
// site of each of A, B, C, Q (-1 for a face plane), si the cell's site.
__device__ inline int side_exact(const PlaneI& A, const PlaneI& B, const PlaneI& C, const PlaneI& Q,
                                 const int* site, int si) {
  i128 bc[3] = {(i128)B.ny * C.nz - (i128)B.nz * C.ny, (i128)B.nz * C.nx - (i128)B.nx * C.nz,
                (i128)B.nx * C.ny - (i128)B.ny * C.nx};
  i128 ca[3] = {(i128)C.ny * A.nz - (i128)C.nz * A.ny, (i128)C.nz * A.nx - (i128)C.nx * A.nz,
                (i128)C.nx * A.ny - (i128)C.ny * A.nx};
  i128 ab[3] = {(i128)A.ny * B.nz - (i128)A.nz * B.ny, (i128)A.nz * B.nx - (i128)A.nx * B.nz,
                (i128)A.nx * B.ny - (i128)A.ny * B.nx};
  I256 W = i256_add(i256_add(i256_mul(i256(A.nx), i256(bc[0])), i256_mul(i256(A.ny), i256(bc[1]))),
                    i256_mul(i256(A.nz), i256(bc[2])));
  int sw = i256_sign(W);
  if (sw == 0) return 2;
  const long long qn[3] = {Q.nx, Q.ny, Q.nz};
  I256 s = i256_mul(i256(Q.d), W);
  for (int k = 0; k < 3; ++k) {
    I256 Xk = i256_add(i256_add(i256_mul(i256(A.d), i256(bc[k])), i256_mul(i256(B.d), i256(ca[k]))),
                       i256_mul(i256(C.d), i256(ab[k])));
    s = i256_add(s, i256_neg(i256_mul(i256(qn[k]), Xk)));  // X = -(...)
  }
  if (i256_sign(s) != 0) return i256_sign(s) * sw;
  // cofactors of the offsets of A, B, C, Q in the raw value
  I256 cof[4];
  const i128* rows[3] = {bc, ca, ab};
  for (int p = 0; p < 3; ++p) {
    I256 t = i256_add(i256_add(i256_mul(i256(qn[0]), i256(rows[p][0])), i256_mul(i256(qn[1]), i256(rows[p][1]))),
                      i256_mul(i256(qn[2]), i256(rows[p][2])));
    cof[p] = i256_neg(t);
  }
  cof[3] = W;
  I256 ci = {{0, 0, 0, 0}};  // coefficient of eps_i: every bisector's cofactor
  for (int p = 0; p < 4; ++p)
    if (site[p] >= 0) ci = i256_add(ci, cof[p]);
  int best = i256_sign(ci) != 0 ? si : 0x7fffffff, best_sign = i256_sign(ci);
  for (int p = 0; p < 4; ++p)  // coefficient of eps_j(P): -c_P (the four planes' sites are distinct)
    if (site[p] >= 0 && site[p] < best && i256_sign(cof[p]) != 0) {
      best = site[p];
      best_sign = -i256_sign(cof[p]);
    }
  return best_sign * sw;
}

// ---------------------------------------------------------------------------------------------------------------
// Plane construction from a tet (4 vertices, absolute float coordinates on the 2^-20 grid) and sites (x,y,z,r).
// Local frame: origin at tet vertex 0.  Face f is the face opposite vertex f, normal pointing inwards.
// ---------------------------------------------------------------------------------------------------------------
RPD_HD inline long long grid_int(float v) { return (long long)(v * 1048576.0f); }

RPD_HD inline PlaneI face_planeI(const float4* tv, int f) {
  int o0 = (f == 0) ? 1 : 0;
  int o1 = (f <= 1) ? 2 : 1;
  int o2 = (f <= 2) ? 3 : 2;
  long long Ox = grid_int(tv[0].x), Oy = grid_int(tv[0].y), Oz = grid_int(tv[0].z);
  long long px = grid_int(tv[o0].x) - Ox, py = grid_int(tv[o0].y) - Oy, pz = grid_int(tv[o0].z) - Oz;
  long long ux = grid_int(tv[o1].x) - grid_int(tv[o0].x), uy = grid_int(tv[o1].y) - grid_int(tv[o0].y),
            uz = grid_int(tv[o1].z) - grid_int(tv[o0].z);
  long long wx = grid_int(tv[o2].x) - grid_int(tv[o0].x), wy = grid_int(tv[o2].y) - grid_int(tv[o0].y),
            wz = grid_int(tv[o2].z) - grid_int(tv[o0].z);
  long long vx = grid_int(tv[f].x) - grid_int(tv[o0].x), vy = grid_int(tv[f].y) - grid_int(tv[o0].y),
            vz = grid_int(tv[f].z) - grid_int(tv[o0].z);
  long long nx = uy * wz - uz * wy, ny = uz * wx - ux * wz, nz = ux * wy - uy * wx;
  if ((i128)nx * vx + (i128)ny * vy + (i128)nz * vz < 0) {
    nx = -nx;
    ny = -ny;
    nz = -nz;
  }
  PlaneI P;
  P.nx = nx;
  P.ny = ny;
  P.nz = nz;
  P.d = -((i128)nx * px + (i128)ny * py + (i128)nz * pz);
  return P;
}

// The same plane in FP64 and float units: the normal (|n| < 2^44 grid units, scaled by 2^-40) is exact and the offset
// (|d| < 2^66 grid units, scaled by 2^-60) is rounded once: its high part times 2^32 and its low 32 bits are both
// exact doubles, so their sum is the single rounding. The FP64 filters rely on this (every input coefficient exact or
// once rounded).
RPD_HD inline double i128_to_double(i128 v) {
  const long long hi = (long long)(v >> 32);  // |v| < 2^85 keeps hi exact in a double
  const unsigned long long lo = (unsigned long long)(v & (i128)0xffffffffull);
  return ldexp((double)hi, 32) + (double)lo;
}
RPD_HD inline Plane<double> face_plane64(const float4* tv, int f) {
  const PlaneI P = face_planeI(tv, f);
  return Plane<double>{ldexp((double)P.nx, -40), ldexp((double)P.ny, -40), ldexp((double)P.nz, -40),
                       ldexp(i128_to_double(P.d), -60)};
}

// power distance of the local origin o to site s, exact in FP64 (all values multiples of 2^-40, < 2^6)
RPD_HD inline double pow_origin64(const float4& s, const float4& o) {
  double ax = (double)s.x - o.x, ay = (double)s.y - o.y, az = (double)s.z - o.z;
  return ax * ax + ay * ay + az * az - (double)s.w * s.w;
}

// bisector of site i against site j (kept side: d_i <= d_j), exact coefficients in FP64
RPD_HD inline Plane<double> bisector64(const float4& si, const float4& sj, const float4& o) {
  return Plane<double>{2.0 * ((double)si.x - sj.x), 2.0 * ((double)si.y - sj.y), 2.0 * ((double)si.z - sj.z),
                       pow_origin64(sj, o) - pow_origin64(si, o)};
}

__device__ inline PlaneI bisectorI(const float4& si, const float4& sj, const float4& o) {
  long long Ox = grid_int(o.x), Oy = grid_int(o.y), Oz = grid_int(o.z);
  long long ix = grid_int(si.x), iy = grid_int(si.y), iz = grid_int(si.z), ir = grid_int(si.w);
  long long jx = grid_int(sj.x), jy = grid_int(sj.y), jz = grid_int(sj.z), jr = grid_int(sj.w);
  long long Di = (ix - Ox) * (ix - Ox) + (iy - Oy) * (iy - Oy) + (iz - Oz) * (iz - Oz) - ir * ir;
  long long Dj = (jx - Ox) * (jx - Ox) + (jy - Oy) * (jy - Oy) + (jz - Oz) * (jz - Oz) - jr * jr;
  PlaneI P;
  P.nx = 2 * (ix - jx);
  P.ny = 2 * (iy - jy);
  P.nz = 2 * (iz - jz);
  P.d = (i128)(Dj - Di);
  return P;
}

template <typename T>
__device__ inline Plane<T> round_plane(const Plane<double>& p) {
  return normalise(Plane<T>{(T)p.nx, (T)p.ny, (T)p.nz, (T)p.d});
}

// ---------------------------------------------------------------------------------------------------------------
// Topology word of one vertex: three plane ids and, for each, the neighbour slot across the edge formed by the two
// OTHER planes (moving along that edge away from the plane).
// ---------------------------------------------------------------------------------------------------------------
struct Topo32 {  // plane ids < 32 (5 bits), slots < 16 (4 bits)
  typedef unsigned W;
  __device__ static int plane(W w, int e) { return (w >> (5 * e)) & 31; }
  __device__ static int nb(W w, int e) { return (w >> (15 + 4 * e)) & 15; }
  __device__ static W make(int p0, int p1, int p2, int n0, int n1, int n2) {
    return (W)p0 | ((W)p1 << 5) | ((W)p2 << 10) | ((W)n0 << 15) | ((W)n1 << 19) | ((W)n2 << 23);
  }
  __device__ static W set_nb(W w, int e, int n) {
    int sh = 15 + 4 * e;
    return (w & ~((W)15 << sh)) | ((W)n << sh);
  }
};
struct Topo64 {  // plane ids < 1024 (10 bits), slots < 256 (8 bits)
  typedef unsigned long long W;
  __device__ static int plane(W w, int e) { return (int)((w >> (10 * e)) & 1023); }
  __device__ static int nb(W w, int e) { return (int)((w >> (32 + 8 * e)) & 255); }
  __device__ static W make(int p0, int p1, int p2, int n0, int n1, int n2) {
    return (W)p0 | ((W)p1 << 10) | ((W)p2 << 20) | ((W)n0 << 32) | ((W)n1 << 40) | ((W)n2 << 48);
  }
  __device__ static W set_nb(W w, int e, int n) {
    int sh = 32 + 8 * e;
    return (w & ~((W)255 << sh)) | ((W)n << sh);
  }
};

template <typename T>
struct Coord4;
template <>
struct Coord4<float> {
  typedef float4 type;
};
template <>
struct Coord4<double> {
  struct __attribute__((aligned(16))) type {
    double x, y, z, w;
  };
};

// vertex storage with a per-thread stride (LDS slices, stride = threads per block) or contiguous (global scratch)
// (slot indices are masked to the capacity, or clamped below it when it is not a power of two, so that every access
// stays inside the thread's slice; live slots are always below the capacity)
template <int VCAP>
__device__ __forceinline__ int vslot(int k) {
  return (VCAP & (VCAP - 1)) == 0 ? (k & (VCAP - 1)) : min(k, VCAP - 1);
}
template <typename T, typename Topo, int VCAP>
struct Store {
  typename Coord4<T>::type* c;
  typename Topo::W* w;
  int stride;
  __device__ typename Coord4<T>::type get(int k) const { return c[vslot<VCAP>(k) * stride]; }
  __device__ void put(int k, T x, T y, T z, T F) {
    typename Coord4<T>::type v;
    v.x = x;
    v.y = y;
    v.z = z;
    v.w = F;
    c[vslot<VCAP>(k) * stride] = v;
  }
  __device__ typename Topo::W topo(int k) const { return w[vslot<VCAP>(k) * stride]; }
  __device__ void set_topo(int k, typename Topo::W t) { w[vslot<VCAP>(k) * stride] = t; }
  __device__ static typename Topo::W with_F(typename Topo::W t, T) { return t; }  // F is stored with the coordinates
  __device__ void bind(void* coords, typename Topo::W* topo_words, int lane, int nthreads) {
    c = reinterpret_cast<typename Coord4<T>::type*>(coords) + lane;
    w = topo_words + lane;
    stride = nthreads;
  }
  static constexpr size_t coord_bytes(int nthreads) { return sizeof(typename Coord4<T>::type) * VCAP * nthreads; }
};

// The FP32 polytopes of the fast kernel in 16 bytes per vertex: x and y as a pair and z in separate [slot][lane]
// planes, the topology word, and in its five free bits the vertex's error bound F rounded up to a power of two
// between 2^-40 and 2^-10 (code 31: infinite, every test on the vertex goes to FP64). Rounding F up only makes the
// FP32 filter more cautious, so every sign it certifies is still right.
__device__ inline unsigned encode_F(float F) {
  if (!(F <= 0x1p-10f)) return 31u;  // also infinite and NaN
  if (F <= 0x1p-40f) return 0u;
  const unsigned b = __float_as_uint(F);
  const int e = (int)((b >> 23) & 255u) - 127;                 // F = 1.m x 2^e, normal here
  return (unsigned)(((b & 0x7fffffu) ? e + 1 : e) + 40);        // ceil(log2 F) + 40, in [1, 30]
}
__device__ inline float decode_F(unsigned code) {
  return code == 31u ? INFINITY : __uint_as_float((code + 87u) << 23);  // 2^(code - 40)
}
template <int VCAP>
struct StoreP {
  float2* xy;  // [VCAP][stride]
  float* zz;   // [VCAP][stride]
  unsigned* w;
  int stride;
  __device__ float4 get(int k) const {
    const int o = vslot<VCAP>(k) * stride;
    const float2 p = xy[o];
    return make_float4(p.x, p.y, zz[o], decode_F(w[o] >> 27));
  }
  __device__ void put(int k, float x, float y, float z, float) {  // F travels in the topology word (with_F)
    const int o = vslot<VCAP>(k) * stride;
    xy[o] = make_float2(x, y);
    zz[o] = z;
  }
  __device__ unsigned topo(int k) const { return w[vslot<VCAP>(k) * stride]; }
  __device__ void set_topo(int k, unsigned t) { w[vslot<VCAP>(k) * stride] = t; }
  __device__ static unsigned with_F(unsigned t, float F) { return (t & 0x07ffffffu) | (encode_F(F) << 27); }
  __device__ void bind(void* coords, unsigned* topo_words, int lane, int nthreads) {
    xy = reinterpret_cast<float2*>(coords) + lane;
    zz = reinterpret_cast<float*>(reinterpret_cast<float2*>(coords) + VCAP * nthreads) + lane;
    w = topo_words + lane;
    stride = nthreads;
  }
  static constexpr size_t coord_bytes(int nthreads) { return (sizeof(float2) + sizeof(float)) * VCAP * nthreads; }
};
template <typename T, typename Topo, int VCAP>
struct StoreOf {
  typedef Store<T, Topo, VCAP> type;
};
template <int VCAP>
struct StoreOf<float, Topo32, VCAP> {  // Topo32 leaves bits 27..31 free
  typedef StoreP<VCAP> type;
};

__device__ inline int ctz_mask(unsigned m) { return __builtin_ctz(m); }
__device__ inline int ctz_mask(unsigned long long m) { return __builtin_ctzll(m); }

// ---------------------------------------------------------------------------------------------------------------
// Environment of one tet: planes by id (0..3 faces, 4+c the bisector against candidate c), site ids, weights.
// ---------------------------------------------------------------------------------------------------------------
struct TetEnv {
  const float4* tv;      // 4 vertices (absolute)
  float4 o;              // vertex 0: the origin of the tet-local frame
  const double4* face64;  // the tet's 4 face planes in FP64 (normal exact, offset rounded once)
  const float4* sites;   // candidate site data, indexed through cidx
  const int* sid;        // site ids, indexed through cidx
  const unsigned char* cidx8;  // candidate -> index into sites/sid (fast path)
  const int* cidx32;     // candidate -> index (slow path)
  const float4* csite;   // the first ncs candidates' sites by candidate position (slow path: on chip), or nullptr
  int ncs;
  int ci;                // candidate position of the piece's own site
  float4 si;             // own site
  int site_i;            // own site id

  __device__ int cand_index(int c) const { return cidx8 ? (int)cidx8[c] : cidx32[c]; }
  __device__ float4 cand_site(int c) const { return c < ncs ? csite[c] : sites[cand_index(c)]; }
  __device__ int cand_id(int c) const { return sid ? sid[cand_index(c)] : cand_index(c); }
  __device__ int plane_site(int p) const { return p < 4 ? -1 : cand_id(p - 4); }

  __device__ Plane<double> plane64(int p) const {
    if (p < 4) {
      const double4 f = face64[p];
      return Plane<double>{f.x, f.y, f.z, f.w};
    }
    return bisector64(si, cand_site(p - 4), o);
  }
  __device__ PlaneI planeI(int p) const {
    if (p < 4) return face_planeI(tv, p);
    return bisectorI(si, cand_site(p - 4), o);
  }
  template <typename T>
  __device__ Plane<T> planeT(int p) const;
};

// FP32 planes are rounded from the FP64 ones on every use (face planes included: the FP64 face planes are read
// through the caches, which keeps the per-workgroup LDS of the fast kernel to its polytopes)
template <>
__device__ inline Plane<float> TetEnv::planeT<float>(int p) const {
  return round_plane<float>(plane64(p));
}
template <>
__device__ inline Plane<double> TetEnv::planeT<double>(int p) const {
  return normalise(plane64(p));
}

// carrier weight numerator L/k of an element given the tet-face planes among its defining planes, as a 4-bit mask
// (faces f are opposite vertex f; local edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) -> 0..5):
// no face: tet interior (L); one face f: that face; two faces: the edge joining the two vertices neither face
// excludes; three faces: their common vertex
__device__ inline int pair_index(int a, int b) {  // a < b
  return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}
__device__ inline long long w_mask(unsigned fm, const unsigned* nu, long long L) {
  const int nf = __builtin_popcount(fm);
  if (nf == 0) return L;
  if (nf == 1) return nu[10 + __builtin_ctz(fm)];
  const unsigned rest = ~fm & 15u;
  if (nf == 2) {
    int a = __builtin_ctz(rest), b = 31 - __builtin_clz(rest);
    return nu[4 + pair_index(a, b)];
  }
  return nu[__builtin_ctz(rest)];
}
__device__ inline unsigned face_bit(int p) { return p < 4 ? (1u << p) : 0u; }
__device__ inline long long w_vertex(int p0, int p1, int p2, const unsigned* nu, long long L) {
  return w_mask(face_bit(p0) | face_bit(p1) | face_bit(p2), nu, L);
}
__device__ inline long long w_edge(int p0, int p1, const unsigned* nu, long long L) {
  return w_mask(face_bit(p0) | face_bit(p1), nu, L);
}

// ---------------------------------------------------------------------------------------------------------------
// hash tables (open addressing, linear probing)
// ---------------------------------------------------------------------------------------------------------------
__device__ inline unsigned hslot(unsigned long long key, unsigned mask) {  // 64-bit finaliser: every key bit mixes
  unsigned long long x = key;
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return (unsigned)x & mask;
}
__device__ inline int ht_insert(const HashTab& h, unsigned long long key, int* status) {
  unsigned s = hslot(key, h.mask);
  for (unsigned probe = 0; probe <= h.mask; ++probe) {
    // most pieces find their element's key present: a plain read first (a stale empty read only costs the atomic)
    const unsigned long long seen = h.keys[s];
    if (seen == key) return (int)s;
    if (seen == EMPTY_KEY) {
      const unsigned long long prev = atomicCAS(&h.keys[s], EMPTY_KEY, key);
      if (prev == EMPTY_KEY || prev == key) return (int)s;
    }
    s = (s + 1) & h.mask;
  }
  atomicOr(status, ST_TABLE_FULL);
  return -1;
}
__device__ inline int ht_find(const HashTab& h, unsigned long long key) {
  unsigned s = hslot(key, h.mask);
  for (unsigned probe = 0; probe <= h.mask; ++probe) {
    unsigned long long k = h.keys[s];
    if (k == key) return (int)s;
    if (k == EMPTY_KEY) return -1;
    s = (s + 1) & h.mask;
  }
  return -1;
}

__device__ inline int node_insert(const NodeTab& h, unsigned long long key, int* status) {
  unsigned s = hslot(key, h.mask);
  for (unsigned probe = 0; probe <= h.mask; ++probe) {
    unsigned long long prev = atomicCAS(&h.rec[s].key, EMPTY_KEY, key);
    if (prev == EMPTY_KEY || prev == key) return (int)s;
    s = (s + 1) & h.mask;
  }
  atomicOr(status, ST_TABLE_FULL);
  return -1;
}
__device__ inline int node_find(const NodeTab& h, unsigned long long key) {
  unsigned s = hslot(key, h.mask);
  for (unsigned probe = 0; probe <= h.mask; ++probe) {
    unsigned long long k = h.rec[s].key;
    if (k == key) return (int)s;
    if (k == EMPTY_KEY) return -1;
    s = (s + 1) & h.mask;
  }
  return -1;
}

__device__ inline unsigned long long node_key(int kind, int elem, int t) {
  return ((unsigned long long)kind << 62) | ((unsigned long long)(unsigned)elem << 32) | (unsigned)t;
}
__device__ inline int node_kind(unsigned long long key) { return (int)(key >> 62); }
__device__ inline int node_elem(unsigned long long key) { return (int)((key >> 32) & 0x3fffffffull); }

// ---------------------------------------------------------------------------------------------------------------
// Per-plane scratch of the clipper (pairing of new vertices; first vertex of each face during emission): entry p is
// 0 or (slot + 1), and every entry is 0 between operations. MemTab keeps it in memory (any number of planes);
// RegTab in five registers (plane ids < 32, slots < 16: four words of 4-bit slots and a word of fifth bits).
// ---------------------------------------------------------------------------------------------------------------
struct MemTab {
  unsigned char* base;
  int stride;
  __device__ __forceinline__ int get(int q) const { return base[q * stride]; }
  __device__ __forceinline__ void set(int q, int v) { base[q * stride] = (unsigned char)v; }
  __device__ __forceinline__ void clear(int np) {
    for (int q = 0; q < np; ++q) base[q * stride] = 0;
  }
};
struct RegTab {
  unsigned w0, w1, w2, w3, hi;
  __device__ void clear(int) { w0 = w1 = w2 = w3 = hi = 0u; }
  __device__ int get(int q) const {
    const unsigned w = q < 8 ? w0 : q < 16 ? w1 : q < 24 ? w2 : w3;
    return (int)(((w >> ((q & 7) * 4)) & 15u) | (((hi >> q) & 1u) << 4));
  }
  __device__ void set(int q, int v) {
    const int sh = (q & 7) * 4;
    const unsigned keep = ~(15u << sh), put = ((unsigned)v & 15u) << sh;
    if (q < 8) w0 = (w0 & keep) | put;
    else if (q < 16) w1 = (w1 & keep) | put;
    else if (q < 24) w2 = (w2 & keep) | put;
    else w3 = (w3 & keep) | put;
    hi = (hi & ~(1u << q)) | (((unsigned)v >> 4) << q);
  }
};

// ---------------------------------------------------------------------------------------------------------------
// The clipper: one convex piece P = t & {clipped half-spaces}, vertices in a Store, live slots in a mask.
// ---------------------------------------------------------------------------------------------------------------
enum { CLIP_OK = 0, CLIP_EMPTY = 1, CLIP_DEFER = 2, CLIP_FULL = 3 };  // DEFER: undecided predicate; FULL: out of vertex slots

template <typename T, typename Topo, typename Mask, int VCAP, bool EXACT, typename Tab>
struct Clipper {
  typedef typename Topo::W W;
  typename StoreOf<T, Topo, VCAP>::type st;
  Tab tab;  // per plane id: 0 or (slot + 1); all zero between operations
  Mask live;
  TetEnv env;
  const ShapeArgs* a;
  unsigned flags;
  int np;  // plane ids in use: 4 faces + candidates
  int n64, nex;

  __device__ static Mask bit(int k) { return (Mask)1 << k; }

  __device__ void init_tet() {
    const float4 o = env.o;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      T x = (T)(env.tv[v].x - o.x), y = (T)(env.tv[v].y - o.y), z = (T)(env.tv[v].z - o.z);
      // the three faces through vertex v (all but face v), ascending; across the edge formed by two of them
      // lies the tet vertex with the third one's index
      const int p0 = (v == 0) ? 1 : 0, p1 = (v <= 1) ? 2 : 1, p2 = (v <= 2) ? 3 : 2;
      const T F = exact_point_F(x, y, z);
      st.put(v, x, y, z, F);
      st.set_topo(v, st.with_F(Topo::make(p0, p1, p2, p0, p1, p2), F));
    }
    live = (Mask)15;
  }

  // exact-or-FP64 decision for vertex k against plane q; 0 means undecided here (defer)
  __device__ int resolve(int k, int q) {
    W w = st.topo(k);
    int pa = Topo::plane(w, 0), pb = Topo::plane(w, 1), pc = Topo::plane(w, 2);
    if (!(flags & RPD_FORCE_EXACT)) {
      ++n64;
      int s = side64(env.plane64(pa), env.plane64(pb), env.plane64(pc), env.plane64(q));
      if (s) return s;
    }
    if (!EXACT) return 0;
    ++nex;
    const int site[4] = {env.plane_site(pa), env.plane_site(pb), env.plane_site(pc), env.plane_site(q)};
    int s = side_exact(env.planeI(pa), env.planeI(pb), env.planeI(pc), env.planeI(q), site, env.site_i);
    if (s == 0 || s == 2) {
      atomicOr(a->status, ST_DEGENERATE);
      return -1;
    }
    return s;
  }

  __device__ void pair_up(int p, int s, W& nw, int pos_in_new) {
    int prev = tab.get(p);
    if (prev == 0) {
      tab.set(p, s + 1);
      return;
    }
    tab.set(p, 0);
    int s1 = prev - 1;
    nw = Topo::set_nb(nw, pos_in_new, s1);
    W w1 = st.topo(s1);
    // in s1 = (pa1, pb1, q): the edge (p, q) is opposite the other one of pa1/pb1
    int pos1 = (Topo::plane(w1, 0) == p) ? 1 : 0;
    st.set_topo(s1, Topo::set_nb(w1, pos1, s));
  }

  __device__ int clip(int q, const Plane<T>& P) {
    Mask out = 0;
    const bool force = (flags & (RPD_FORCE_FP64 | RPD_FORCE_EXACT)) != 0;
    for (Mask m = live; m; m &= m - 1) {
      int k = ctz_mask(m);
      typename Coord4<T>::type v = st.get(k);
      int s = force ? 0 : side_fast(P, v.x, v.y, v.z, v.w);
      if (s == 0) s = resolve(k, q);
      if (s == 0) return CLIP_DEFER;
      if (s < 0) out |= bit(k);
    }
    if (!out) return CLIP_OK;
    if (out == live) {
      live = 0;
      return CLIP_EMPTY;
    }
    const Mask full = (VCAP >= 8 * (int)sizeof(Mask)) ? ~(Mask)0 : ((bit(VCAP)) - 1);
    Mask kept = live & ~out;
    Mask freem = ~kept & full;
    Mask added = 0;
    for (Mask m = kept; m; m &= m - 1) {
      int k = ctz_mask(m);
      W w = st.topo(k);
      bool changed = false;
      for (int e = 0; e < 3; ++e) {
        int nb = Topo::nb(w, e);
        if (!(out & bit(nb))) continue;
        if (!freem) {  // out of vertex slots: clear the half-done pairing state and give the piece up
          tab.clear(np);
          return CLIP_FULL;
        }
        int s = ctz_mask(freem);
        freem &= freem - 1;
        int pa = Topo::plane(w, (e + 1) % 3), pb = Topo::plane(w, (e + 2) % 3);
        T x, y, z, F;
        make_vertex(env.planeT<T>(pa), env.planeT<T>(pb), P, x, y, z, F);
        W nw = st.with_F(Topo::make(pa, pb, q, 0, 0, k), F);
        st.put(s, x, y, z, F);
        pair_up(pa, s, nw, 1);  // edge (pa, q) is opposite pb (position 1)
        pair_up(pb, s, nw, 0);  // edge (pb, q) is opposite pa (position 0)
        st.set_topo(s, nw);
        w = Topo::set_nb(w, e, s);
        changed = true;
        added |= bit(s);
      }
      if (changed) st.set_topo(k, w);
    }
    live = kept | added;
    return CLIP_OK;
  }
};

}  // namespace rpd
