// Test harness: the library's own plane constructions and FP64 filter (rpd_device.h), compiled for the host so that a
// CPU test can compare them with exact arithmetic. Built by tests/test_host_predicates.py; not part of librpd.
#include "rpd_device.h"

extern "C" {

// tv: 4 vertices (x, y, z) of a positively oriented tet; sites: n sites (x, y, z, r). Plane id p < 4 is face p of the
// tet (opposite vertex p), p >= 4 is the bisector of site si against site p - 4. Returns side64 of plane ids[3] at
// the meet of planes ids[0..2], and the four FP64 planes (nx, ny, nz, d) in planes_out.
int host_side64(const float* tv, const float* sites, int si, const int* ids, double* planes_out) {
  float4 t[4];
  for (int v = 0; v < 4; ++v) t[v] = make_float4(tv[3 * v], tv[3 * v + 1], tv[3 * v + 2], 0.0f);
  const float4 s_i = make_float4(sites[4 * si], sites[4 * si + 1], sites[4 * si + 2], sites[4 * si + 3]);
  rpd::Plane<double> P[4];
  for (int k = 0; k < 4; ++k) {
    const int p = ids[k];
    if (p < 4) {
      P[k] = rpd::face_plane64(t, p);
    } else {
      const float* q = sites + 4 * (p - 4);
      P[k] = rpd::bisector64(s_i, make_float4(q[0], q[1], q[2], q[3]), t[0]);
    }
    planes_out[4 * k] = P[k].nx;
    planes_out[4 * k + 1] = P[k].ny;
    planes_out[4 * k + 2] = P[k].nz;
    planes_out[4 * k + 3] = P[k].d;
  }
  return rpd::side64(P[0], P[1], P[2], P[3]);
}

}  // extern "C"
