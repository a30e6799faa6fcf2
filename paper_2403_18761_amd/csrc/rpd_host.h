// Host-side helpers of librpd (internal): error reporting, device buffers, the prepared mesh.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "rpd.h"
#include "rpd_common.h"

namespace rpd {

// the calling thread's last error message (a fixed buffer: setting it allocates nothing)
void set_error(const char* msg);
inline void set_error(const std::string& msg) { set_error(msg.c_str()); }

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

// Caching device allocator: freed blocks are kept in per-device free lists keyed by their power-of-two size class
// and reused, so repeated rpd_build calls do not pay hipMalloc/hipFree. Memory returns to the runtime only when the
// process ends.
void* pool_alloc(size_t bytes, size_t* cls_bytes, int* device);
void pool_free(void* p, size_t cls_bytes, int device);

// owning device allocation (through the pool)
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int dev = 0;  // the device the block belongs to (its free list)
  DBuf() = default;
  explicit DBuf(size_t n) { alloc(n); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes), dev(o.dev) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    release();
    p = o.p;
    bytes = o.bytes;
    dev = o.dev;
    o.p = nullptr;
    o.bytes = 0;
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) n = 16;
    p = pool_alloc(n, &bytes, &dev);
  }
  void release() {
    if (p) pool_free(p, bytes, dev);
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
  int32_t owner = 0;  // ownership weights
  int device = 0;
  rpd::DBuf tp;    // float4 [4 nt]: vertex coordinates per internal tet
  rpd::DBuf tf;    // double4 [4 nt]: face planes of every internal tet in FP64 (normal exact, offset rounded once)
  rpd::DBuf tn;    // int [4 nt]: neighbour internal tet across local face f
  rpd::DBuf nu;    // unsigned [14 nt]: weight numerators
  rpd::DBuf perm;  // int [nt]: internal -> caller tet index
  rpd::DBuf blk;   // int [nblk + 1]: workgroup blocks over the internal order
  int32_t nblk = 0;
  std::vector<int> hblk;  // host copy of blk
  // Fast-kernel time of every block in the last build that used this mesh: a dispatch-order hint for the next
  // build (heaviest first); never read by any kernel.
  std::mutex cost_mu;
  std::vector<unsigned> blk_cost;
};

namespace rpd {
void mesh_prepare(rpd_mesh* m, const rpd_mesh_desc* d, uint32_t flags, hipStream_t s);
}
