// Host-side helpers of librpd (internal): error reporting, device buffers, the prepared mesh.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rpd.h"
#include "rpd_common.h"

namespace rpd {

void set_error(const std::string& msg);

struct Failure {
  rpd_status code;
  std::string msg;
};

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) throw Failure{RPD_E_NOMEM, std::string(what) + ": out of device memory"};
    throw Failure{RPD_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
  }
}

// owning device allocation
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  explicit DBuf(size_t n) { alloc(n); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    release();
    p = o.p;
    bytes = o.bytes;
    o.p = nullptr;
    o.bytes = 0;
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) n = 16;
    hip_check(hipMalloc(&p, n), "hipMalloc");
    bytes = n;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const {
    return (T*)p;
  }
};

}  // namespace rpd

// the prepared mesh (opaque in the public header)
struct rpd_mesh {
  int32_t nv = 0, nt = 0, n_edges = 0, n_faces = 0;
  int32_t euler = 0, components = 0;
  int64_t L = 1;
  double volume = 0;
  int device = 0;
  rpd::DBuf tp;    // float4 [4 nt]: vertex coordinates per internal tet
  rpd::DBuf tn;    // int [4 nt]: neighbour internal tet across local face f
  rpd::DBuf nu;    // unsigned [14 nt]: weight numerators
  rpd::DBuf perm;  // int [nt]: internal -> caller tet index
};

namespace rpd {
void mesh_prepare(rpd_mesh* m, const rpd_mesh_desc* d, uint32_t flags, hipStream_t s);
}
