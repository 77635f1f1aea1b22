// Internal declarations of the bemfmm library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "bemfmm.h"

namespace bem {

struct Error : std::runtime_error {
  bem_status code;
  int64_t element;
  Error(bem_status c, const std::string& m, int64_t e = -1)
      : std::runtime_error(m), code(c), element(e) {}
};

#define BEM_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      throw ::bem::Error(e_ == hipErrorOutOfMemory ? BEM_E_OOM : BEM_E_HIP, \
                         std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Device allocator of the plan memory: hipMalloc / hipFree, or the caller's
// pair set with bem_set_allocator (process-wide; a buffer keeps the pair it
// was allocated with).
struct AllocHook {
  bem_alloc_fn alloc = nullptr;
  bem_free_fn free = nullptr;
  void* ctx = nullptr;
};
AllocHook current_alloc_hook();

// Owning device buffer.  alloc() keeps the allocation when the new size fits
// (capacity only grows), so per-frequency state re-sized for every wavenumber
// of a sweep does not go back to the allocator each time.
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;    // elements in use
  size_t cap = 0;  // elements allocated
  AllocHook hook{};
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), cap(o.cap), hook(o.hook) { o.p = nullptr; o.n = o.cap = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      cap = o.cap;
      hook = o.hook;
      o.p = nullptr;
      o.n = o.cap = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      if (hook.free) {
        // hipFree waits for the device; a caller's allocator may hand the
        // block out again at once, so wait here before returning it
        (void)hipDeviceSynchronize();
        hook.free(p, cap * sizeof(T), hook.ctx);
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    n = cap = 0;
  }
  void alloc(size_t count) {
    if (p && count <= cap) {
      n = count;
      return;
    }
    release();
    if (count == 0) return;
    hook = current_alloc_hook();
    if (hook.alloc) {
      p = static_cast<T*>(hook.alloc(count * sizeof(T), hook.ctx));
      if (!p) throw Error(BEM_E_OOM, "the allocator set with bem_set_allocator returned NULL");
    } else {
      BEM_HIP(hipMalloc(&p, count * sizeof(T)));
    }
    n = cap = count;
  }
  // Copy a host vector to the device and wait for the copy (setup paths only:
  // the caller's vector may be released right after the call).
  void upload(const std::vector<T>& h, hipStream_t s = nullptr) {
    alloc(h.size());
    if (!h.empty()) {
      BEM_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
      BEM_HIP(hipStreamSynchronize(s));
    }
  }
  size_t bytes() const { return cap * sizeof(T); }
};

// ---------------------------------------------------------------- rules ---
// 1-D rules on [0, 1]: Gauss-Legendre, and Gauss for weight xi.
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);
void gauss_jacobi_xi01(int n, std::vector<double>& x, std::vector<double>& w);

// ------------------------------------------------------------- geometry ---
// Element data in structure-of-arrays form, field f of element e at f*N + e.
enum GeomField {
  G_P0X = 0, G_P0Y, G_P0Z, G_P1X, G_P1Y, G_P1Z, G_P2X, G_P2Y, G_P2Z,
  G_NX, G_NY, G_NZ, G_AREA, G_CX, G_CY, G_CZ, G_NFIELDS
};

// Elements are flat triangles or plane quadrilaterals (Sec. 2.2).  A
// quadrilateral P0 P1 P2 P3 keeps P0, P1, P2 in its own fields, its vertex
// mean as collocation node, the normal along (P2 - P0) x (P3 - P1) and its
// whole area; it is integrated as the two triangles (P0, P1, P2) and
// (P0, P2, P3), the integration records N + 2q and N + 2q + 1 (q its
// quadrilateral index), whose geometry is held in hq with the GeomField
// layout and stride 2 nq.  Integration records j < N are the triangles.
struct Geometry {
  int64_t N = 0;
  std::vector<double> f;  // G_NFIELDS * N
  int64_t nq = 0;               // quadrilaterals
  std::vector<int64_t> qidx;    // element -> quadrilateral index, or -1 (empty: triangles only)
  std::vector<int64_t> hown;    // half record r (record N + r) -> element
  std::vector<double> hq;       // G_NFIELDS * 2 nq: the halves (P0, P1, P2, normal, area, centroid)
  double& at(int field, int64_t e) { return f[field * N + e]; }
  double at(int field, int64_t e) const { return f[field * N + e]; }
  bool is_quad(int64_t e) const { return !qidx.empty() && qidx[e] >= 0; }
  int nv(int64_t e) const { return is_quad(e) ? 4 : 3; }
  // vertex v (0..3) coordinate d of element e; P3 of a quadrilateral is the
  // third vertex of its second half
  double vtx(int v, int d, int64_t e) const {
    return v < 3 ? at(G_P0X + 3 * v + d, e) : hq[(G_P2X + d) * 2 * nq + 2 * qidx[e] + 1];
  }
  // element of integration record j
  int64_t owner(int64_t j) const { return j < N ? j : hown[j - N]; }
};

// Build geometry in the order given by perm (perm[t] = caller index of the
// element at position t).  el: n_el x 4 vertex indices, el[4 e + 3] < 0 for a
// triangle.  Throws BEM_E_MESH on a degenerate element, a quadrilateral that
// is not plane or not convex.
Geometry build_geometry(const double* xyz, int64_t n_nodes, const int32_t* el,
                        int64_t n_el, const std::vector<int64_t>& perm);

// ----------------------------------------------------------------- tree ---
struct Level {
  int64_t nc = 0;
  std::vector<double> z;           // 3 * nc
  std::vector<double> r;           // nc
  std::vector<int64_t> ebeg, eend; // element range in tree order
  std::vector<int64_t> parent;     // cluster index on the level above (-1 at root)
  std::vector<int64_t> cbeg, cend; // children range on the level below
  std::vector<int64_t> il_off, il; // interaction list (CSR)
  std::vector<int64_t> nr_off, nr; // near list (CSR)
};

struct Tree {
  std::vector<Level> lv;        // lv[0] = root level
  std::vector<int64_t> perm;    // tree position -> caller element index
  std::vector<int64_t> inv;     // caller element index -> tree position
};

// Cluster tree of Sec. 3.3.2-3.3.4 on the caller-ordered geometry gc.
Tree build_tree(const Geometry& gc, int levels, double root_edge, int leaf_size,
                double admissibility);

// -------------------------------------------------------- near-field plan ---
// One quadrature item: a (sub-)triangle of source element j integrated with
// an order-m conical rule.  Packed in 64 bits:
//   bits  0..25  j (tree position)
//   bits 26..28  m - 1
//   bits 29..32  subdivision depth
//   bits 33..62  path, two bits per level (child index 0..3), level 0 lowest
struct NearPlan {
  std::vector<int64_t> off;     // per target (tree order), size N+1
  std::vector<int64_t> seg;     // per target 9 offsets: first item of order 1..8, then the end
  std::vector<uint64_t> items;
  int64_t pairs = 0;            // near pairs including self pairs
  int64_t points = 0;           // quadrature points per application
  int max_m = 1;
};

struct QuadParams {
  double eps;
  int m_max;
  int split_on_cap;
  double ratio;
  int max_subdiv;
};

// targets: element positions (tree order); for target t the sources are
// [src_ranges) given by a callback-free CSR: src_off/src_beg/src_end.
// Per-target offsets of the rule-order segments of an item list sorted by order.
void build_segments(NearPlan& P, int64_t N);

NearPlan build_near_plan(const Geometry& g, const QuadParams& q,
                         const std::vector<int64_t>& tgt_src_off,
                         const std::vector<int64_t>& src_beg,
                         const std::vector<int64_t>& src_end,
                         const std::vector<int64_t>& tgt_group);

}  // namespace bem
