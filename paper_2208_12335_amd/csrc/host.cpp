// Host side of the C ABI: validation, spline construction, spatial batching, screening,
// upload, and the call sequences of the entry points declared in include/aims_grid.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <iterator>
#include <map>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "aims_grid.h"
#include "aims_internal.h"
#include "kernels.h"
#include "scf.h"
#include "xc.h"
#include "hartree.h"

using namespace aims;

namespace {

thread_local std::string g_setup_error = "no error";

// Scratch of the allocation-free density update (aims_update_density_noalloc): the two basis
// slabs of one group of batches, in a static device array that every GPU the library runs on
// holds until the process ends.  Host code never passes the array's name to a kernel (in host
// code it names a host-side stand-in); it uses the device address that hipGetSymbolAddress
// returns, taken once per device at set-up with that device current.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kDensityBuckets = 8;   // basis-size classes of 64 functions (the tile-shape buckets)
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// ---------------------------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------------------------
struct Fail {
  aims_status status;
  std::string msg;
};

[[noreturn]] void fail(aims_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Fail{st, buf};
}

void hipchk(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(AIMS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

template <typename F>
void parallel_for(int64_t n, F&& f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 64 || nt == 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next(0);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&] {
      for (int64_t i; (i = next.fetch_add(1)) < n;) f(i);
    });
  for (auto& t : th) t.join();
}

bool finite_all(const double* x, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

// Natural cubic spline through y_k at uniformly spaced abscissae (spacing h): second
// derivatives from the tridiagonal system M_{k-1} + 4 M_k + M_{k+1} = 6 (y_{k+1} - 2 y_k +
// y_{k-1}) / h^2 with M_0 = M_{n-1} = 0, then per interval the coefficients of
// a + b t + c t^2 + d t^3 in t = s - s_k.
void natural_spline(const double* y, int n, double h, double* coef /* [(n-1)][4] */) {
  std::vector<double> M(n, 0.0), cp(n, 0.0), dp(n, 0.0);
  const int m = n - 2;  // unknowns M_1..M_{n-2}
  for (int i = 0; i < m; ++i) {
    const int k = i + 1;
    const double rhs = 6.0 * (y[k + 1] - 2.0 * y[k] + y[k - 1]) / (h * h);
    const double denom = 4.0 - (i > 0 ? cp[i - 1] : 0.0);
    cp[i] = 1.0 / denom;
    dp[i] = (rhs - (i > 0 ? dp[i - 1] : 0.0)) / denom;
  }
  for (int i = m - 1; i >= 0; --i) M[i + 1] = dp[i] - (i + 1 < m ? cp[i] * M[i + 2] : 0.0);
  for (int k = 0; k < n - 1; ++k) {
    coef[4 * k + 0] = y[k];
    coef[4 * k + 1] = (y[k + 1] - y[k]) / h - h * (2.0 * M[k] + M[k + 1]) / 6.0;
    coef[4 * k + 2] = 0.5 * M[k];
    coef[4 * k + 3] = (M[k + 1] - M[k]) / (6.0 * h);
  }
}

// The batch tree of one system.  A node [lo, hi) of batch-ordered points carries a leaf count
// L: the root's is the smallest power of two with L x max_batch >= n (the depth of a plain
// median bisection), each child takes max(1, L / 2), and a node is a batch once L = 1 and it
// holds at most max_batch points.  A node splits at its median, moved to the nearest multiple
// of kSplit points from lo once it holds at least 2 kSplit points (both halves stay non-empty).
// Left children are then multiples of kSplit, so every batch of a system but its last fills
// whole slab rows (kPad points) and whole 64-point FP64 density tiles: no padded point columns
// to evaluate, store or multiply.
constexpr int64_t kSplit = 2 * kPad;
int64_t tree_leaves(int64_t n, int64_t maxb) {
  int64_t L = 1;
  while (L * maxb < n) L <<= 1;
  return L;
}

int64_t split_point(int64_t lo, int64_t hi) {
  const int64_t n = hi - lo;
  int64_t h = n / 2;
  if (n >= 2 * kSplit) h = (h + kSplit / 2) / kSplit * kSplit;
  return lo + h;
}

// Recursive bisection along the longest bounding-box axis at split_point (ties broken by index).
void bisect(const double* xyz, std::vector<int32_t>& idx, int64_t lo, int64_t hi, int64_t L,
            int maxb, std::vector<std::pair<int64_t, int64_t>>& out) {
  if (hi <= lo) return;
  if (L <= 1 && hi - lo <= maxb) {
    out.emplace_back(lo, hi);
    return;
  }
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = lo; i < hi; ++i)
    for (int c = 0; c < 3; ++c) {
      mn[c] = std::min(mn[c], xyz[3 * (int64_t)idx[i] + c]);
      mx[c] = std::max(mx[c], xyz[3 * (int64_t)idx[i] + c]);
    }
  int ax = 0;
  for (int c = 1; c < 3; ++c)
    if (mx[c] - mn[c] > mx[ax] - mn[ax]) ax = c;
  const int64_t mid = split_point(lo, hi);
  std::nth_element(idx.begin() + lo, idx.begin() + mid, idx.begin() + hi, [&](int32_t a, int32_t b) {
    const double ca = xyz[3 * (int64_t)a + ax], cb = xyz[3 * (int64_t)b + ax];
    return ca < cb || (ca == cb && a < b);
  });
  const int64_t Lc = std::max<int64_t>(1, L / 2);
  bisect(xyz, idx, lo, mid, Lc, maxb, out);
  bisect(xyz, idx, mid, hi, Lc, maxb, out);
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged ||
         attr.type == hipMemoryTypeUnified;
}

}  // namespace

// -------------------------------------------------------------------------------------------------
// batch sets and the handle
// -------------------------------------------------------------------------------------------------
// One partition of the (batch-ordered) points into batches, with per-batch screening, the groups
// of batches that share the scratch slabs, and the MFMA tile work list.  The density pass uses
// the partition at max_batch; the H/S pass may use a coarser one (max_batch << merge, i.e. the
// bisection stopped `merge` levels earlier), which trades a few more flops for fewer FP64
// scatter-adds into H.
struct ItemList {
  uint64_t key = 0;                // tile shapes of the list (tile_key)
  std::vector<TileItem> items;
  struct Run {
    int nbn;                       // point blocks of the kernel variant (density), 0 for H
    int64_t i0, i1;
  };
  std::vector<std::vector<Run>> runs;  // per group of batches
  TileItem* d_items = nullptr;
};

struct BatchSet {
  int merge = 0;
  int ratio = 0;                   // > 0: cost-model partition (flop-equivalents per scatter-add)
  bool density = false;            // tile lists for the density kernel (else for the H kernel)
  std::vector<BatchDesc> batches;
  std::vector<int32_t> batch_atoms, batch_acol, batch_cols;
  struct Group {
    int b0, b1;                    // batches
    double flops;                  // sum over the group's batches of 2 n_p n_b^2
  };
  std::vector<Group> groups;
  std::vector<int64_t> sys_batch_range;
  size_t slab_elems = 0;
  double sum_np_nb2 = 0, sum_nb2 = 0;
  std::vector<std::unique_ptr<ItemList>> lists;
  // device copies
  DeviceView dv{};
  int32_t* d_colexp = nullptr;     // int8 form: per batch column, exponents of the two H operands
  int max_nb = 0;                  // largest batch basis count
};

struct aims_grid {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err = "no error";

  int n_sys = 0;
  int n_atoms = 0;
  int64_t n_points = 0;
  int64_t nb_total = 0;
  int64_t mat_total = 0;
  double margin = 1e-2;
  RadialGrid rg{};

  std::vector<double> atom_xyz0;      // setup positions
  bool moved = false;                 // device positions differ from the setup positions
  std::vector<SystemDesc> systems;
  std::vector<int64_t> sys_pt_range, sys_atom_range;
  std::vector<int> sys_max_batch;
  std::vector<std::vector<int>> atom_nfn;     // per system, per atom
  std::vector<std::vector<int>> atom_col0;    // per system, per atom: first basis index
  std::vector<double4> pts_sorted;            // host copy of the batch-ordered points

  BatchSet dens;                              // density partition (merge 0)
  BatchSet dens_na;                           // the same batches grouped for the static scratch
  void* na_scratch = nullptr;                 // device address of `scratch` on this handle's device
  std::string na_error;                       // non-empty: the static scratch cannot hold a batch
  std::vector<std::unique_ptr<BatchSet>> hsets;  // H partitions by merge level (built on demand)
  int h_merge[4] = {1, 2, 2, 1};              // per precision
  int h_ratio[4] = {0, 0, 0, 0};              // per precision: > 0 selects the cost-model H partition
  int d_pblocks[4] = {2, 5, 5, 2};            // per precision: density point-tile cap (int8: 64)
  int persistent[4] = {0, 0, 0, 0};           // per precision: persistent tile launches
  int32_t d_bucket_pblocks[4][kDensityBuckets] = {};   // per precision and basis-size bucket (0 = d_pblocks)
  uint32_t h_tile32[4] = {0, 0, 0, 0};        // per precision: H buckets on 32 x 32 tiles (FP64, FP32)
  int* d_queue = nullptr;                     // 8 work counters per tiled launch of one call
  size_t queue_cap = 0;                       // counters allocated
  int nblk_finish = 64;

  // profiling
  struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double work;
  };
  bool profiling = false;
  bool graph_captured = false;        // a step graph may reference the current scratch
  std::vector<ProfRec> prof_pending;
  int64_t prof_count[6] = {0, 0, 0, 0, 0, 0};
  double prof_ms[6] = {0, 0, 0, 0, 0, 0};
  double prof_work[6] = {0, 0, 0, 0, 0, 0};

  std::vector<void*> owned;           // device allocations
  DeviceView common{};                // device pointers shared by every batch set
  double* d_atom_xyz = nullptr;
  double* d_atom_xyz0 = nullptr;      // set-up positions (restored device to device)
  int* d_pos_flag = nullptr;          // 1 when the last device positions failed the screening check
  unsigned long long* d_dbg = nullptr;  // AIMS_DEBUG: maxima of the symmetry check, 2 per system
  bool pos_async = false;             // this call took positions on the device (outputs checked)
  double* d_n_sorted = nullptr;
  double* d_part = nullptr;
  double* d_et_batch = nullptr;
  float* d_P32 = nullptr;
  uint64_t* d_P8 = nullptr;           // int8 form: digit words of P
  int32_t* d_eP = nullptr;            // int8 form: exponent of each row of P
  int32_t* d_pexp = nullptr;          // int8 form: per point (batch order), exponents of Phi, t Phi
  void* d_slab1 = nullptr;
  void* d_slab2 = nullptr;
  void* d_slab3 = nullptr;            // backward: X = Phi P_b
  void* d_slab4 = nullptr;            // backward: Y = (T Phi) P_b
  size_t slab_cap = 0;                // elements per slab currently allocated
  size_t slab_cap34 = 0;
  double* d_ntmp = nullptr;           // backward: n in caller order (not returned)
  double* d_sums_tmp = nullptr;

  // moving-grid model of each system (total energy gradient)
  std::vector<int32_t> perm_host;            // batch-ordered point -> caller index
  std::vector<char> moving;                  // per system: model set
  std::vector<double> sys_model;             // [n_sys][2]: sigma, partition a
  std::vector<int32_t> owner_host;           // batch order: owner atom (handle-global)
  std::vector<double> wgrid_host;            // batch order: weight before the partition
  std::vector<double> Z_host;                // per handle-global atom
  std::vector<int32_t> pt_sys_host;          // batch order: system of the point
  int32_t* d_owner = nullptr;
  double* d_wgrid = nullptr;
  double* d_Z = nullptr;
  double* d_sys_model = nullptr;
  int32_t* d_sys_natoms = nullptr;
  int32_t* d_pt_sys = nullptr;
  double* d_vmodel = nullptr;                // model potential, caller order
  double* d_dsorted = nullptr;               // kinetic density per point, batch order
  double* d_gpt = nullptr;                   // point-motion sums, batch order [n][3]
  // wave-per-point force kernel: 1 / (a R_bc) tables, batch ranges and per-range slots
  double* d_xc_part = nullptr;               // per-block partial sums of the xc kernels
  // Hartree multipole expansion: per system radial grid, per point owner / radial node
  int hartree_lmax = -1;
  std::vector<int> h_K;                      // [n_sys] radial nodes (0 = not set)
  std::vector<double> h_rmap;                // [n_sys]
  std::vector<int32_t> h_owner;              // [n_points] global atom, batch order
  std::vector<int32_t> h_node;               // [n_points] radial node, batch order
  bool h_ready = false;
  HartreeDev hd;
  int dm_iterations = 0;                     // purification products of the last system
  bool force_thread_path = false;           // AIMS_FORCES_THREAD_PATH=1: thread-per-point kernel
  bool debug = false;                        // AIMS_DEBUG=1: check every index table on the host
  bool gf_ready = false;
  int gf_k = 0;
  int gf_nranges = 0;
  ForceRange* d_franges = nullptr;
  double* d_inv_aR = nullptr;
  int64_t* d_pair_off = nullptr;
  double* d_fpart = nullptr;
  int64_t* d_fpart_off = nullptr;
  int32_t* d_fnrange = nullptr;

  DmSolver dm;                                // density-matrix step (rocBLAS handle, work matrices)

  ~aims_grid() {
    (void)hipSetDevice(device);
    dm_release(dm);
    for (void* p : owned) (void)hipFree(p);
  }

  void* alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    const char* inj = getenv("AIMS_FAIL_ALLOC");
    if (inj && atoi(inj) != 0) fail(AIMS_ERR_OOM, "device allocation of %zu bytes failed (injected)", bytes);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(AIMS_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    owned.push_back(p);
    return p;
  }
  void release(void* p) {
    auto it = std::find(owned.begin(), owned.end(), p);
    if (it != owned.end()) {
      (void)hipFree(p);
      owned.erase(it);
    }
  }
  template <typename T>
  T* upload(const std::vector<T>& v) {
    T* p = (T*)alloc(v.size() * sizeof(T));
    if (!v.empty())
      hipchk(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
    return p;
  }
};

namespace {

// ---------------------------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------------------------
void validate_system(const aims_system* s, int k) {
  if (!s) fail(AIMS_ERR_ARG, "system %d: null aims_system", k);
  if (s->n_atoms < 1) fail(AIMS_ERR_ARG, "system %d: n_atoms must be >= 1", k);
  if (!s->atom_xyz || !s->atom_species || !s->species_nshell || !s->shell_l || !s->shell_R ||
      !s->shell_K)
    fail(AIMS_ERR_ARG, "system %d: null array", k);
  if (s->n_species < 1) fail(AIMS_ERR_ARG, "system %d: n_species must be >= 1", k);
  if (s->n_points < 0) fail(AIMS_ERR_ARG, "system %d: n_points < 0", k);
  if (s->n_points > 0 && (!s->pt_xyz || !s->pt_w)) fail(AIMS_ERR_ARG, "system %d: null points", k);
  if (s->n_points > (int64_t)INT32_MAX / 2) fail(AIMS_ERR_UNSUPPORTED, "system %d: too many points", k);
  if (s->max_batch < 1 || s->max_batch > kMaxBatch)
    fail(AIMS_ERR_UNSUPPORTED, "system %d: max_batch must be in [1, %d]", k, kMaxBatch);
  if (s->n_log < 4) fail(AIMS_ERR_ARG, "system %d: n_log must be >= 4", k);
  if (!(s->r0 > 0.0) || !(s->rc > s->r0) || !std::isfinite(s->rc))
    fail(AIMS_ERR_ARG, "system %d: need 0 < r0 < rc", k);
  int nsh = 0;
  for (int i = 0; i < s->n_species; ++i) {
    if (s->species_nshell[i] < 1 || s->species_nshell[i] > kMaxShells)
      fail(AIMS_ERR_UNSUPPORTED, "system %d: species %d has %d shells (1..%d supported)", k, i,
           s->species_nshell[i], kMaxShells);
    nsh += s->species_nshell[i];
  }
  for (int i = 0; i < nsh; ++i)
    if (s->shell_l[i] < 0 || s->shell_l[i] > kLmax)
      fail(AIMS_ERR_UNSUPPORTED, "system %d: shell %d has l = %d (0..3 supported)", k, i, s->shell_l[i]);
  for (int a = 0; a < s->n_atoms; ++a)
    if (s->atom_species[a] < 0 || s->atom_species[a] >= s->n_species)
      fail(AIMS_ERR_ARG, "system %d: atom %d has species %d out of range", k, a, s->atom_species[a]);
  {
    // the tiled kernels address a system's P with 32-bit element offsets (n_basis^2 < 2^32)
    std::vector<int64_t> nfn(s->n_species, 0);
    for (int i = 0, sh = 0; i < s->n_species; ++i)
      for (int j = 0; j < s->species_nshell[i]; ++j, ++sh) nfn[i] += 2 * s->shell_l[sh] + 1;
    int64_t nb = 0;
    for (int a = 0; a < s->n_atoms; ++a) nb += nfn[s->atom_species[a]];
    if (nb > kMaxBasis)
      fail(AIMS_ERR_UNSUPPORTED, "system %d: %lld basis functions (at most %d)", k, (long long)nb,
           kMaxBasis);
  }
  if (!finite_all(s->atom_xyz, 3 * (size_t)s->n_atoms)) fail(AIMS_ERR_ARG, "system %d: non-finite atom_xyz", k);
  if (!finite_all(s->shell_R, (size_t)nsh * s->n_log) || !finite_all(s->shell_K, (size_t)nsh * s->n_log))
    fail(AIMS_ERR_ARG, "system %d: non-finite radial table", k);
  if (s->n_points > 0 && (!finite_all(s->pt_xyz, 3 * (size_t)s->n_points) || !finite_all(s->pt_w, (size_t)s->n_points)))
    fail(AIMS_ERR_ARG, "system %d: non-finite grid", k);
}

size_t scratch_budget_elems() {
  // elements per slab (two slabs); 8 GiB total in FP64 by default: fewer, larger groups
  // (fewer launch tails) measured faster, the gain levelling off once a 1.1M-point, 1445-function
  // step fits one group (8 GiB), and 288 GB leaves room for it
  double mb = 8192.0;
  if (const char* e = getenv("AIMS_SCRATCH_MB")) mb = std::max(16.0, atof(e));
  return (size_t)(mb * 1024.0 * 1024.0 / 16.0);
}

// Segments of the batch-ordered points of one system: the nodes of its batch tree with leaf
// count <= Lm holding at most Lm x maxb points (Lm = 1: the batches; Lm = 2^m: the tree
// stopped m levels earlier).  Because the set-up bisection already ordered the points, every
// segment is a contiguous range.
void segments(int64_t lo, int64_t hi, int64_t L, int64_t maxb, int64_t Lm,
              std::vector<std::pair<int64_t, int64_t>>& out) {
  if (hi <= lo) return;
  if (L <= Lm && hi - lo <= maxb * Lm) {
    out.emplace_back(lo, hi);
    return;
  }
  const int64_t mid = split_point(lo, hi);
  const int64_t Lc = std::max<int64_t>(1, L / 2);
  segments(lo, mid, Lc, maxb, Lm, out);
  segments(mid, hi, Lc, maxb, Lm, out);
}

// Cost-model partition of one system for the H pass.  Every node of the set-up bisection (a
// contiguous point range) may become one H batch of up to 4 x max_batch points; its relevant
// atoms are the union of its children's (an atom is relevant to a range iff it is relevant to
// one of its points), so the density batches' exact screening gives every node's basis size
// n_b.  A node of n points costs 2 n n_b^2 flops plus `ratio` flop-equivalents for each of its
// n_b^2 FP64 scatter-adds into H; a bottom-up pass keeps a node whole when that is cheaper than
// the best partitions of its two halves.
struct NodeCost {
  double cost;
  std::vector<int32_t> atoms;                         // sorted, system-local
  std::vector<std::pair<int64_t, int64_t>> segs;      // chosen H batches of the subtree
};

NodeCost cost_partition(int64_t lo, int64_t hi, int64_t L, int64_t maxb, int64_t cap, double ratio,
                        const std::map<int64_t, const std::vector<int32_t>*>& leaf_atoms,
                        const std::vector<int>& nfn) {
  NodeCost r;
  r.cost = 0.0;
  if (hi <= lo) return r;
  const bool leaf = L <= 1 && hi - lo <= maxb;
  if (leaf) {
    auto it = leaf_atoms.find(lo);
    if (it != leaf_atoms.end()) r.atoms = *it->second;
  } else {
    const int64_t mid = split_point(lo, hi);
    const int64_t Lc = std::max<int64_t>(1, L / 2);
    NodeCost a = cost_partition(lo, mid, Lc, maxb, cap, ratio, leaf_atoms, nfn);
    NodeCost b = cost_partition(mid, hi, Lc, maxb, cap, ratio, leaf_atoms, nfn);
    std::set_union(a.atoms.begin(), a.atoms.end(), b.atoms.begin(), b.atoms.end(),
                   std::back_inserter(r.atoms));
    r.cost = a.cost + b.cost;
    r.segs = std::move(a.segs);
    r.segs.insert(r.segs.end(), b.segs.begin(), b.segs.end());
  }
  double nb = 0;
  for (int32_t at : r.atoms) nb += nfn[at];
  const double own = 2.0 * (double)(hi - lo) * nb * nb + ratio * nb * nb;
  if (leaf || (hi - lo <= cap && own <= r.cost)) {
    r.cost = own;
    r.segs.assign(1, {lo, hi});
  }
  return r;
}

size_t form_groups(BatchSet& bs, size_t budget);
void upload_set(aims_grid* g, BatchSet& bs);

void build_set(aims_grid* g, BatchSet& bs, int merge, bool density, int ratio = 0) {
  bs.merge = merge;
  bs.ratio = ratio;
  bs.density = density;
  const double reach = g->rg.rc + g->margin;
  for (int k = 0; k < g->n_sys; ++k) {
    const int64_t base = g->sys_pt_range[2 * k], end = g->sys_pt_range[2 * k + 1];
    std::vector<std::pair<int64_t, int64_t>> segs;
    if (ratio > 0 && !density) {
      // leaves: the density batches of this system and their screened atoms
      const int a0k = g->systems[k].atom_off;
      std::vector<std::vector<int32_t>> leaf_lists;
      std::map<int64_t, const std::vector<int32_t>*> leaf_atoms;
      leaf_lists.reserve(g->dens.batches.size());
      for (const BatchDesc& d : g->dens.batches) {
        if (d.sys != k) continue;
        std::vector<int32_t> at(g->dens.batch_atoms.begin() + d.atom_off,
                                g->dens.batch_atoms.begin() + d.atom_off + d.n_atoms);
        for (auto& x : at) x -= a0k;
        std::sort(at.begin(), at.end());
        leaf_lists.push_back(std::move(at));
        leaf_atoms[d.pt_off] = &leaf_lists.back();
      }
      const int64_t maxb = g->sys_max_batch[k];
      segs = cost_partition(base, end, tree_leaves(end - base, maxb), maxb, maxb << 2, (double)ratio,
                            leaf_atoms, g->atom_nfn[k]).segs;
    } else {
      const int64_t maxb = g->sys_max_batch[k];
      segments(base, end, tree_leaves(end - base, maxb), maxb, (int64_t)1 << merge, segs);
    }
    const int nseg = (int)segs.size();
    const int a0 = g->systems[k].atom_off;
    const int na = (int)g->atom_nfn[k].size();
    std::vector<std::vector<int32_t>> rel(nseg);
    parallel_for(nseg, [&](int64_t b) {
      const int64_t lo = segs[b].first, hi = segs[b].second;
      double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
      for (int64_t i = lo; i < hi; ++i) {
        const double4& p = g->pts_sorted[i];
        const double c3[3] = {p.x, p.y, p.z};
        for (int c = 0; c < 3; ++c) {
          mn[c] = std::min(mn[c], c3[c]);
          mx[c] = std::max(mx[c], c3[c]);
        }
      }
      double cen[3], rad2 = 0;
      for (int c = 0; c < 3; ++c) {
        cen[c] = 0.5 * (mn[c] + mx[c]);
        rad2 += 0.25 * (mx[c] - mn[c]) * (mx[c] - mn[c]);
      }
      const double rad = std::sqrt(rad2);
      for (int a = 0; a < na; ++a) {
        const double* A = g->atom_xyz0.data() + 3 * (size_t)(a0 + a);
        const double dc = std::sqrt((A[0] - cen[0]) * (A[0] - cen[0]) + (A[1] - cen[1]) * (A[1] - cen[1]) +
                                    (A[2] - cen[2]) * (A[2] - cen[2]));
        if (dc - rad >= reach) continue;
        bool hit = false;
        for (int64_t i = lo; i < hi && !hit; ++i) {
          const double4& p = g->pts_sorted[i];
          const double d2 = (p.x - A[0]) * (p.x - A[0]) + (p.y - A[1]) * (p.y - A[1]) +
                            (p.z - A[2]) * (p.z - A[2]);
          hit = d2 < reach * reach;
        }
        if (hit) rel[b].push_back(a);
      }
    });
    for (int b = 0; b < nseg; ++b) {
      // each batch's column list starts on a multiple of 4 entries (16-byte index loads)
      while (bs.batch_cols.size() % 4) bs.batch_cols.push_back(0);
      BatchDesc d{};
      d.pt_off = (int32_t)segs[b].first;
      d.n_p = (int32_t)(segs[b].second - segs[b].first);
      d.atom_off = (int32_t)bs.batch_atoms.size();
      d.n_atoms = (int32_t)rel[b].size();
      d.col_off = (int32_t)bs.batch_cols.size();
      d.sys = k;
      d.ldp = round_up(d.n_p, kPad);
      int col = 0;
      for (int a : rel[b]) {
        bs.batch_atoms.push_back(a0 + a);
        bs.batch_acol.push_back(col);
        for (int f = 0; f < g->atom_nfn[k][a]; ++f) bs.batch_cols.push_back(g->atom_col0[k][a] + f);
        col += g->atom_nfn[k][a];
      }
      d.n_b = col;
      bs.batches.push_back(d);
      bs.sum_np_nb2 += (double)d.n_p * d.n_b * d.n_b;
      bs.sum_nb2 += (double)d.n_b * d.n_b;
    }
  }
  // tail padding: index loads of a K chunk may read up to 31 entries past a batch's list
  bs.batch_cols.insert(bs.batch_cols.end(), 32, 0);
  if ((int64_t)bs.batch_cols.size() > (int64_t)INT32_MAX) fail(AIMS_ERR_UNSUPPORTED, "too many batch columns");

  form_groups(bs, scratch_budget_elems());
  // batch range of each system (batches are in system order)
  bs.sys_batch_range.assign(2 * (size_t)g->n_sys, 0);
  const int nB = (int)bs.batches.size();
  for (int s = 0, b = 0; s < g->n_sys; ++s) {
    bs.sys_batch_range[2 * s] = b;
    while (b < nB && bs.batches[b].sys == s) ++b;
    bs.sys_batch_range[2 * s + 1] = b;
  }
  upload_set(g, bs);
}

// Groups of consecutive batches whose slabs fit `budget` elements per slab, and the slab offset
// of each batch within its group.  Returns the largest single-batch need (elements).
size_t form_groups(BatchSet& bs, size_t budget) {
  bs.groups.clear();
  bs.slab_elems = 0;
  size_t largest = 0;
  BatchSet::Group cur{0, 0, 0.0};
  size_t used = 0;
  const int nB = (int)bs.batches.size();
  for (int b = 0; b < nB; ++b) {
    BatchDesc& d = bs.batches[b];
    const size_t need = (size_t)round_up(d.n_b, 32) * d.ldp;
    if (used > 0 && used + need > budget) {
      cur.b1 = b;
      bs.groups.push_back(cur);
      cur = BatchSet::Group{b, b, 0.0};
      used = 0;
    }
    cur.flops += 2.0 * d.n_p * (double)d.n_b * d.n_b;
    bs.max_nb = std::max(bs.max_nb, d.n_b);
    d.slab_off = (int64_t)used;
    used += need;
    largest = std::max(largest, need);
    bs.slab_elems = std::max(bs.slab_elems, used);
  }
  cur.b1 = nB;
  if (cur.b1 > cur.b0) bs.groups.push_back(cur);
  return largest;
}

// Device copies of a batch set's tables; the handle's slabs grow to the set's largest group.
void upload_set(aims_grid* g, BatchSet& bs) {
  bs.dv = g->common;
  bs.dv.batches = g->upload(bs.batches);
  bs.dv.batch_atoms = g->upload(bs.batch_atoms);
  bs.dv.batch_acol = g->upload(bs.batch_acol);
  bs.dv.batch_cols = g->upload(bs.batch_cols);
  bs.dv.sys_batch_range = g->upload(bs.sys_batch_range);
  if (bs.slab_elems > g->slab_cap) {
    // A step graph captured earlier may still reference the smaller scratch, so it then stays
    // allocated until the handle is destroyed (as it does while the stream is being captured).
    // Otherwise it is released, once the stream has drained, before the larger one is taken.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (g->stream) hipchk(hipStreamIsCapturing(g->stream, &cap), "capture status");
    if (!g->graph_captured && cap == hipStreamCaptureStatusNone && g->d_slab1) {
      hipchk(hipStreamSynchronize(g->stream), "synchronize before releasing scratch");
      g->release(g->d_slab1);
      g->release(g->d_slab2);
      g->d_slab1 = g->d_slab2 = nullptr;
    }
    g->slab_cap = 0;
    g->d_slab1 = g->alloc(bs.slab_elems * sizeof(double));
    g->d_slab2 = g->alloc(bs.slab_elems * sizeof(double));
    g->slab_cap = bs.slab_elems;
  }
}

// Point blocks (of 32) of the density tile for a batch of n_p points under a cap: the batch is
// cut into ceil(n_p / (32 cap)) tiles of equal block count, at least 2 blocks each.
int density_nbn(int n_p, int cap) {
  const int blocks = (n_p + 31) / 32;
  const int tiles = (blocks + cap - 1) / cap;
  return std::max(2, (blocks + tiles - 1) / tiles);
}

// Tile work list of a batch set: square 64 x 64 tiles for the H kernel, (64 rows x 32 nbn
// points) tiles for the density kernel, grouped per kernel variant within each batch group.
// AIMS_DEBUG: every index the kernels read through a batch set's tables, checked on the host
// against the buffers it addresses (points, atoms, basis columns, slabs, the work list's tiles).
void debug_check(const aims_grid* g, const BatchSet& bs, const ItemList* L, const char* what) {
  auto bad = [&](const char* m, int64_t b) {
    fail(AIMS_ERR_ARG, "internal table check (%s): %s at batch %lld", what, m, (long long)b);
  };
  const int64_t nB = (int64_t)bs.batches.size();
  for (int64_t b = 0; b < nB; ++b) {
    const BatchDesc& d = bs.batches[b];
    if (d.sys < 0 || d.sys >= g->n_sys) bad("system index", b);
    const int64_t p0 = g->sys_pt_range[2 * d.sys], p1 = g->sys_pt_range[2 * d.sys + 1];
    if (d.n_p < 0 || d.pt_off < p0 || d.pt_off + (int64_t)d.n_p > p1) bad("point range", b);
    if (d.ldp != round_up(d.n_p, kPad)) bad("slab row length", b);
    if (d.atom_off < 0 || d.atom_off + (int64_t)d.n_atoms > (int64_t)bs.batch_atoms.size()) bad("atom range", b);
    if (d.col_off < 0 || d.col_off % 4 || d.col_off + (int64_t)d.n_b + 32 > (int64_t)bs.batch_cols.size())
      bad("column range", b);
    const int64_t a0 = g->sys_atom_range[2 * d.sys], a1 = g->sys_atom_range[2 * d.sys + 1];
    int col = 0;
    for (int k = 0; k < d.n_atoms; ++k) {
      const int32_t at = bs.batch_atoms[d.atom_off + k];
      if (at < a0 || at >= a1) bad("atom index", b);
      if (bs.batch_acol[d.atom_off + k] != col) bad("atom column", b);
      col += g->atom_nfn[d.sys][at - a0];
    }
    if (col != d.n_b) bad("basis count", b);
    for (int j = 0; j < d.n_b; ++j) {
      const int32_t c = bs.batch_cols[d.col_off + j];
      if (c < 0 || c >= g->systems[d.sys].nb) bad("basis column", b);
    }
    if (d.slab_off < 0 || d.slab_off + (int64_t)round_up(d.n_b, 32) * d.ldp > (int64_t)bs.slab_elems)
      bad("slab extent", b);
  }
  for (const auto& gr : bs.groups)
    if (gr.b0 < 0 || gr.b1 > nB || gr.b0 >= gr.b1) bad("group range", gr.b0);
  if (!L) return;
  const bool hlist = (L->key >> 63) != 0;
  for (size_t gi = 0; gi < L->runs.size(); ++gi)
    for (const auto& run : L->runs[gi])
      for (int64_t i = run.i0; i < run.i1; ++i) {
        const TileItem& it = L->items[i];
        if (it.batch < bs.groups[gi].b0 || it.batch >= bs.groups[gi].b1) bad("tile outside its group", it.batch);
        const BatchDesc& d = bs.batches[it.batch];
        const int rows = hlist ? (run.nbn ? 32 : 64) : kTile;
        const int pts = hlist ? rows : 32 * run.nbn;
        if (it.ti < 0 || it.ti * rows >= d.n_b) bad("tile row", it.batch);
        if (it.tj < 0 || it.tj * pts >= (hlist ? d.n_b : d.n_p)) bad("tile column", it.batch);
      }
}

// Tile shapes by (points, basis count) bucket.  The density pass buckets its batches by basis
// count, kDensityBuckets classes of 64 functions (the last open-ended); each class has its own
// point-tile cap.  The H / S pass buckets by basis count class and by whether the last 64-wide
// tile row is at most half full (n_b mod 64 in 1..32); each bucket runs 64 x 64 or 32 x 32
// tiles.  The batches of one bucket run as one launch per group of batches.
int density_bucket(int n_b) { return std::min(kDensityBuckets - 1, std::max(0, (n_b - 1) / 64)); }
int h_bucket(int n_b) {
  const int r = n_b % 64;
  return 2 * std::min(kDensityBuckets - 1, std::max(0, (n_b - 1) / 64)) + (r != 0 && r <= 32 ? 1 : 0);
}

// Key of a work list: density -- the default cap (4 bits) and the per-bucket caps (4 bits each,
// 0 = default); H -- the mask of 32 x 32 buckets, tagged by bit 63.
uint64_t density_key(int pblocks, const int32_t* bucket_pblocks) {
  uint64_t k = (uint64_t)pblocks;
  for (int b = 0; b < kDensityBuckets; ++b) k |= (uint64_t)(bucket_pblocks ? bucket_pblocks[b] : 0) << (4 + 4 * b);
  return k;
}
uint64_t h_key(uint32_t mask) { return (1ull << 63) | mask; }

ItemList& tile_list(aims_grid* g, BatchSet& bs, uint64_t key, bool counters = true) {
  for (auto& l : bs.lists)
    if (l->key == key) return *l;
  std::unique_ptr<ItemList> L(new ItemList());
  L->key = key;
  const bool hlist = (key >> 63) != 0;
  for (const auto& gr : bs.groups) {
    std::vector<std::vector<TileItem>> per(6);
    for (int b = gr.b0; b < gr.b1; ++b) {
      const BatchDesc& d = bs.batches[b];
      if (hlist) {
        const bool t32 = (key >> h_bucket(d.n_b)) & 1u;
        const int te = t32 ? 32 : 64;
        const int tb = (d.n_b + te - 1) / te;
        for (int ti = 0; ti < tb; ++ti)
          for (int tj = 0; tj < tb; ++tj) per[t32 ? 1 : 0].push_back(TileItem{b, (int16_t)ti, (int16_t)tj});
      } else {
        const int tb = (d.n_b + kTile - 1) / kTile;
        const int cap_b = (int)((key >> (4 + 4 * density_bucket(d.n_b))) & 15u);
        const int nbn = density_nbn(d.n_p, cap_b ? cap_b : (int)(key & 15u));
        const int tp = (d.n_p + 32 * nbn - 1) / (32 * nbn);
        for (int ti = 0; ti < tb; ++ti)
          for (int tj = 0; tj < tp; ++tj) per[nbn].push_back(TileItem{b, (int16_t)ti, (int16_t)tj});
      }
    }
    std::vector<ItemList::Run> runs;
    for (int v = 0; v < 6; ++v) {
      if (per[v].empty()) continue;
      runs.push_back(ItemList::Run{v, (int64_t)L->items.size(), (int64_t)(L->items.size() + per[v].size())});
      L->items.insert(L->items.end(), per[v].begin(), per[v].end());
    }
    L->runs.push_back(runs);
  }
  if ((int64_t)L->items.size() > INT32_MAX) fail(AIMS_ERR_UNSUPPORTED, "too many tiles");
  if (g->debug) debug_check(g, bs, L.get(), hlist ? "H work list" : "density work list");
  L->d_items = g->upload(L->items);
  size_t launches = 0;
  for (const auto& r : L->runs) launches += r.size();
  if (counters && 8 * launches > g->queue_cap) {
    g->d_queue = (int*)g->alloc(8 * launches * sizeof(int));
    g->queue_cap = 8 * launches;
  }
  bs.lists.push_back(std::move(L));
  return *bs.lists.back();
}

// The density list with one cap for every bucket (the allocation-free path, set-up) and the
// lists a precision's tuning selects.
ItemList& items_for(aims_grid* g, BatchSet& bs, int pblocks, bool counters = true) {
  return tile_list(g, bs, density_key(pblocks, nullptr), counters);
}
uint64_t dens_key_of(const aims_grid* g, int prec) {
  if (prec == AIMS_INT8X7) return density_key(2, nullptr);     // 64-point tiles only
  return density_key(g->d_pblocks[prec], g->d_bucket_pblocks[prec]);
}
uint64_t h_key_of(const aims_grid* g, int prec) {
  return h_key(prec == AIMS_FP64 || prec == AIMS_FP32 ? g->h_tile32[prec] : 0u);
}

BatchSet& hset(aims_grid* g, int merge, int ratio = 0) {
  if (ratio > 0) merge = 0;
  for (auto& p : g->hsets)
    if (p->merge == merge && p->ratio == ratio) return *p;
  std::unique_ptr<BatchSet> bs(new BatchSet());
  build_set(g, *bs, merge, false, ratio);
  tile_list(g, *bs, h_key(0));
  g->hsets.push_back(std::move(bs));
  return *g->hsets.back();
}

// Point-tile cap of the allocation-free density update's work list (fixed: that call never
// builds a list).
constexpr int kNoAllocPblocks = 2;

// Device address of the static scratch on the current device, looked up once per device.
void* noalloc_scratch_address(int device) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    fail(AIMS_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  }
  addr[device] = p;
  return p;
}

// The density batches grouped so that one group's two slabs fit the static scratch (half each,
// sized for FP64 values, so the narrower forms fit too), with their own slab offsets and tile
// list.  Only the batch descriptors differ from the density set on the device.
void build_noalloc_set(aims_grid* g) {
  BatchSet& src = g->dens;
  BatchSet& bs = g->dens_na;
  bs.merge = 0;
  bs.density = true;
  bs.batches = src.batches;
  bs.batch_atoms = src.batch_atoms;     // host copies (the device tables are the density set's)
  bs.batch_acol = src.batch_acol;
  bs.batch_cols = src.batch_cols;
  bs.sys_batch_range = src.sys_batch_range;
  bs.sum_np_nb2 = src.sum_np_nb2;
  bs.sum_nb2 = src.sum_nb2;
  const size_t budget = kNoAllocScratchBytes / 2 / sizeof(double);
  const size_t largest = form_groups(bs, budget);
  g->na_scratch = noalloc_scratch_address(g->device);
  if (largest > budget) {
    char buf[256];
    snprintf(buf, sizeof(buf), "a batch needs %zu bytes per basis slab, above the %zu of the "
             "static scratch of aims_update_density_noalloc", largest * sizeof(double), budget * sizeof(double));
    g->na_error = buf;
    return;
  }
  bs.dv = src.dv;
  bs.dv.batches = g->upload(bs.batches);
  items_for(g, bs, kNoAllocPblocks, false);
}

aims_grid* build(const aims_system* sys, int n_sys, int device, void* stream) {
  if (n_sys < 1) fail(AIMS_ERR_ARG, "n_sys must be >= 1");
  if (n_sys > 65535) fail(AIMS_ERR_UNSUPPORTED, "at most 65535 systems per handle (grid y extent)");
  if (!sys) fail(AIMS_ERR_ARG, "null system array");
  for (int k = 0; k < n_sys; ++k) validate_system(&sys[k], k);
  for (int k = 1; k < n_sys; ++k)
    if (sys[k].n_log != sys[0].n_log || sys[k].r0 != sys[0].r0 || sys[k].rc != sys[0].rc)
      fail(AIMS_ERR_ARG, "all systems of one handle must share n_log, r0 and rc");

  std::unique_ptr<aims_grid> g(new aims_grid());
  g->device = device;
  g->stream = (hipStream_t)stream;
  g->n_sys = n_sys;
  g->margin = sys[0].screen_margin > 0 ? sys[0].screen_margin : 1e-2;
  const int n_log = sys[0].n_log;
  g->rg.s0 = std::log(sys[0].r0);
  g->rg.h = (std::log(sys[0].rc) - std::log(sys[0].r0)) / (n_log - 1);
  g->rg.inv_h = 1.0 / g->rg.h;
  g->rg.rc = sys[0].rc;
  g->rg.n_log = n_log;
  if (const char* e = getenv("AIMS_H_MERGE")) {
    const int m = std::max(0, std::min(4, atoi(e)));
    for (int p = 0; p < 3; ++p) g->h_merge[p] = m;
  }
  if (const char* e = getenv("AIMS_FORCES_THREAD_PATH")) g->force_thread_path = atoi(e) != 0;
  if (const char* e = getenv("AIMS_DEBUG")) g->debug = atoi(e) != 0;

  // ---- species, splines, atoms ----------------------------------------------------------
  std::vector<SpeciesDesc> species;
  std::vector<int32_t> shell_l;
  std::vector<int32_t> shell_fexp;   // per shell: balancing exponent of the int8 form
  std::vector<int32_t> fn_fexp;      // per global basis function: the same, per function
  std::vector<double> spline64;
  std::vector<int32_t> atom_species, atom_sys;
  g->atom_nfn.resize(n_sys);
  g->atom_col0.resize(n_sys);
  for (int k = 0; k < n_sys; ++k) {
    const aims_system& s = sys[k];
    const int sp_base = (int)species.size();
    int sh_off = 0;
    for (int i = 0; i < s.n_species; ++i) {
      SpeciesDesc sd{};
      sd.nshell = s.species_nshell[i];
      sd.shell_l_off = (int)shell_l.size();
      sd.spline_off = (int64_t)spline64.size();
      int nfn = 0, lmax = 0;
      for (int j = 0; j < sd.nshell; ++j) {
        const int l = s.shell_l[sh_off + j];
        shell_l.push_back(l);
        // power of two near the shell's largest |R Y_lm| (largest tabulated |R| times
        // sqrt((2l + 1) / (4 pi))): the int8 form divides the density pass's basis values by it
        // and multiplies the matching columns of P by it, an exact rescaling that evens out the
        // digit scales of a point's functions
        double rmax = 0.0;
        for (int kk = 0; kk < n_log; ++kk) rmax = std::max(rmax, std::fabs(s.shell_R[(size_t)(sh_off + j) * n_log + kk]));
        int ex = 0;
        if (rmax > 0.0) (void)std::frexp(rmax * std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI)), &ex);
        shell_fexp.push_back(ex);
        nfn += 2 * l + 1;
        lmax = std::max(lmax, l);
      }
      sd.nfn = nfn;
      sd.lmax = lmax;
      // coefficients at [(k * nshell + j) * 8 + c], c = R a..d, K a..d
      std::vector<double> cR((size_t)(n_log - 1) * 4), cK((size_t)(n_log - 1) * 4);
      spline64.resize(spline64.size() + (size_t)(n_log - 1) * sd.nshell * 8);
      double* base = spline64.data() + sd.spline_off;
      for (int j = 0; j < sd.nshell; ++j) {
        natural_spline(s.shell_R + (size_t)(sh_off + j) * n_log, n_log, g->rg.h, cR.data());
        natural_spline(s.shell_K + (size_t)(sh_off + j) * n_log, n_log, g->rg.h, cK.data());
        for (int kk = 0; kk < n_log - 1; ++kk)
          for (int c = 0; c < 4; ++c) {
            base[((size_t)kk * sd.nshell + j) * 8 + c] = cR[4 * kk + c];
            base[((size_t)kk * sd.nshell + j) * 8 + 4 + c] = cK[4 * kk + c];
          }
      }
      species.push_back(sd);
      sh_off += sd.nshell;
    }
    SystemDesc sdsc{};
    sdsc.mat_off = g->mat_total;
    sdsc.row_off = g->nb_total;
    sdsc.atom_off = g->n_atoms;
    int nb = 0;
    for (int a = 0; a < s.n_atoms; ++a) {
      const int gs = sp_base + s.atom_species[a];
      atom_species.push_back(gs);
      atom_sys.push_back(k);
      g->atom_col0[k].push_back(nb);
      g->atom_nfn[k].push_back(species[gs].nfn);
      nb += species[gs].nfn;
      for (int j = 0; j < species[gs].nshell; ++j)
        for (int m = 0; m < 2 * shell_l[species[gs].shell_l_off + j] + 1; ++m)
          fn_fexp.push_back(shell_fexp[species[gs].shell_l_off + j]);
      for (int c = 0; c < 3; ++c) g->atom_xyz0.push_back(s.atom_xyz[3 * a + c]);
    }
    sdsc.nb = nb;
    g->systems.push_back(sdsc);
    g->sys_atom_range.push_back(g->n_atoms);
    g->n_atoms += s.n_atoms;
    g->sys_atom_range.push_back(g->n_atoms);
    g->sys_max_batch.push_back(s.max_batch);
    g->nb_total += nb;
    g->mat_total += (int64_t)nb * nb;
  }
  std::vector<float> spline32(spline64.begin(), spline64.end());

  // ---- points: batch order from the recursive bisection -----------------------------------
  std::vector<int32_t> perm;
  int64_t caller_base = 0;
  for (int k = 0; k < n_sys; ++k) {
    const aims_system& s = sys[k];
    std::vector<int32_t> idx(s.n_points);
    for (int64_t i = 0; i < s.n_points; ++i) idx[i] = (int32_t)i;
    std::vector<std::pair<int64_t, int64_t>> segs;
    bisect(s.pt_xyz, idx, 0, s.n_points, tree_leaves(s.n_points, s.max_batch), s.max_batch, segs);
    g->sys_pt_range.push_back((int64_t)g->pts_sorted.size());
    for (int64_t i = 0; i < s.n_points; ++i) {
      const int32_t q = idx[i];
      g->pts_sorted.push_back(make_double4(s.pt_xyz[3 * q], s.pt_xyz[3 * q + 1], s.pt_xyz[3 * q + 2], s.pt_w[q]));
      perm.push_back((int32_t)(caller_base + q));
    }
    g->sys_pt_range.push_back((int64_t)g->pts_sorted.size());
    caller_base += s.n_points;
  }
  g->n_points = (int64_t)g->pts_sorted.size();
  g->perm_host = perm;

  // ---- upload of the shared state, then the density partition ---------------------------
  hipchk(hipSetDevice(device), "hipSetDevice");
  hipchk(prepare_launch_configs(), "occupancy query");

  hipchk(prepare_launch_configs_i8(), "occupancy query");
  DeviceView& dv = g->common;
  dv.systems = g->upload(g->systems);
  dv.pts = g->upload(g->pts_sorted);
  dv.perm = g->upload(perm);
  g->d_atom_xyz = g->upload(g->atom_xyz0);
  g->d_atom_xyz0 = g->upload(g->atom_xyz0);
  g->d_pos_flag = g->upload(std::vector<int>(1, 0));
  if (g->debug) g->d_dbg = (unsigned long long*)g->alloc(2 * g->systems.size() * sizeof(unsigned long long));
  dv.atom_xyz = g->d_atom_xyz;
  dv.atom_species = g->upload(atom_species);
  dv.atom_sys = g->upload(atom_sys);
  dv.species = g->upload(species);
  dv.shell_l = g->upload(shell_l);
  dv.shell_fexp = g->upload(shell_fexp);
  dv.fn_fexp = g->upload(fn_fexp);
  dv.spline64 = g->upload(spline64);
  dv.spline32 = g->upload(spline32);
  dv.sys_pt_range = g->upload(g->sys_pt_range);
  dv.rg = g->rg;
  dv.n_sys = n_sys;
  build_set(g.get(), g->dens, 0, true);
  g->d_n_sorted = (double*)g->alloc(std::max<int64_t>(1, g->n_points) * sizeof(double));
  g->d_part = (double*)g->alloc((size_t)n_sys * g->nblk_finish * 2 * sizeof(double));
  g->d_et_batch = (double*)g->alloc(std::max<size_t>(1, g->dens.batches.size()) * sizeof(double));
  for (int p = 0; p < 3; ++p) items_for(g.get(), g->dens, g->d_pblocks[p]);
  build_noalloc_set(g.get());
  g->d_P32 = (float*)g->alloc(std::max<int64_t>(1, g->mat_total) * sizeof(float));
  // the H partitions of the default merge levels
  for (int p = 0; p < 3; ++p) hset(g.get(), g->h_merge[p], g->h_ratio[p]);
  return g.release();
}

// ---------------------------------------------------------------------------------------------
// per-call helpers
// ---------------------------------------------------------------------------------------------
// A caller array the call reads or writes: `bytes` of device memory from p, all inside one
// allocation (hipMemGetAddressRange), so that a short buffer is refused on the host instead of
// being overrun on the device.  Zero-length arrays are never touched and not checked.
void require_device(const void* p, const char* name, size_t bytes) {
  if (bytes == 0) return;
  if (!p) fail(AIMS_ERR_ARG, "%s is NULL", name);
  if (!is_device_ptr(p)) fail(AIMS_ERR_ARG, "%s must be device memory", name);
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess || !base) {
    (void)hipGetLastError();
    fail(AIMS_ERR_ARG, "%s: no device allocation found", name);
  }
  const size_t off = (size_t)((const char*)p - (const char*)base);
  if (off > size || size - off < bytes)
    fail(AIMS_ERR_ARG, "%s: %zu bytes needed, the allocation holds %zu from this pointer", name,
         bytes, off > size ? (size_t)0 : size - off);
}

void check_prec(aims_precision p) {
  if (p != AIMS_FP64 && p != AIMS_FP32 && p != AIMS_BF16X3 && p != AIMS_INT8X7)
    fail(AIMS_ERR_ARG, "unknown precision %d", (int)p);
}

// The forward passes only (density, H, S) have the sliced integer form.
void forward_only(aims_precision p, const char* what) {
  if (p == AIMS_INT8X7) fail(AIMS_ERR_UNSUPPORTED, "%s: AIMS_INT8X7 serves the density, H and S passes only", what);
}

// Positions for this call: NULL = setup positions (restored on the device).  A device array is
// copied and checked on the device, with no host synchronisation (so the call can be captured):
// if any atom is not finite or moved more than screen_margin, the call's outputs become NaN
// (poison_outputs) and aims_positions_status reports AIMS_ERR_STALE.  A host array is checked on
// the host before any launch.
void set_positions(aims_grid* g, const double* xyz) {
  const size_t n = 3 * (size_t)g->n_atoms;
  g->pos_async = false;
  if (!xyz) {
    if (g->moved) {
      hipchk(hipMemcpyAsync(g->d_atom_xyz, g->d_atom_xyz0, n * sizeof(double), hipMemcpyDeviceToDevice,
                            g->stream), "restore positions");
      hipchk(launch_positions_check(g->d_atom_xyz, g->d_atom_xyz0, g->n_atoms, g->margin, g->d_pos_flag,
                                    g->stream), "position check");
      g->moved = false;
    }
    return;
  }
  if (is_device_ptr(xyz)) {
    require_device(xyz, "atom_xyz", n * sizeof(double));
    hipchk(hipMemcpyAsync(g->d_atom_xyz, xyz, n * sizeof(double), hipMemcpyDeviceToDevice, g->stream),
           "positions");
    hipchk(launch_positions_check(g->d_atom_xyz, g->d_atom_xyz0, g->n_atoms, g->margin, g->d_pos_flag,
                                  g->stream), "position check");
    g->moved = true;
    g->pos_async = true;
    return;
  }
  std::vector<double> h(xyz, xyz + n);
  for (int a = 0; a < g->n_atoms; ++a) {
    double d2 = 0;
    for (int c = 0; c < 3; ++c) {
      if (!std::isfinite(h[3 * a + c])) fail(AIMS_ERR_ARG, "non-finite position of atom %d", a);
      const double d = h[3 * a + c] - g->atom_xyz0[3 * a + c];
      d2 += d * d;
    }
    if (d2 > g->margin * g->margin)
      fail(AIMS_ERR_STALE, "atom %d moved %.3g bohr since setup (margin %.3g)", a, std::sqrt(d2), g->margin);
  }
  hipchk(hipMemcpyAsync(g->d_atom_xyz, h.data(), n * sizeof(double), hipMemcpyHostToDevice, g->stream), "positions");
  hipchk(hipStreamSynchronize(g->stream), "positions");
  hipchk(launch_positions_check(g->d_atom_xyz, g->d_atom_xyz0, g->n_atoms, g->margin, g->d_pos_flag,
                                g->stream), "position check");
  g->moved = true;
}

// AIMS_DEBUG: a density matrix that is not symmetric is refused.  Every formula here takes
// P = P^T: the backward's X = Phi P and Y = (T Phi) P, the forces and the density gradient are
// the derivatives only for a symmetric P, and an asymmetric P's kinetic term depends on which
// index a kernel contracts first.  Checked on the device per system (max |P - P^T| <= 1e-12
// max |P|, every entry finite), with one synchronisation; skipped while the stream is being
// captured.
void debug_check_symmetric(aims_grid* g, const double* P, const char* name) {
  if (!g->debug || !g->d_dbg) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(g->stream, &cs) != hipSuccess) (void)hipGetLastError();
  if (cs != hipStreamCaptureStatusNone) return;
  const size_t ns = g->systems.size();
  for (size_t k = 0; k < ns; ++k)
    hipchk(launch_asym_max(P + g->systems[k].mat_off, g->systems[k].nb, g->d_dbg + 2 * k, g->stream),
           "AIMS_DEBUG symmetry check");
  std::vector<unsigned long long> h(2 * ns);
  hipchk(hipMemcpyAsync(h.data(), g->d_dbg, h.size() * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, g->stream), "AIMS_DEBUG symmetry check");
  hipchk(hipStreamSynchronize(g->stream), "AIMS_DEBUG symmetry check");
  for (size_t k = 0; k < ns; ++k) {
    double a, m;
    std::memcpy(&a, &h[2 * k], sizeof(double));
    std::memcpy(&m, &h[2 * k + 1], sizeof(double));
    if (!(a <= 1e-12 * m))
      fail(AIMS_ERR_ARG, "AIMS_DEBUG: %s of system %zu is not symmetric (max|P - P^T| = %.3e, max|P| = %.3e)",
           name, k, a, m);
  }
}

// Outputs of a call that took device positions: NaN if those failed the check.
void poison_outputs(aims_grid* g, double* x, size_t n) {
  if (g->pos_async && x) hipchk(launch_poison(x, n, g->d_pos_flag, g->stream), "position check");
}

enum { kProfPhi = 0, kProfDensity = 1, kProfHS = 2, kProfBackward = 3, kProfFinish = 4, kProfOperands = 5 };
const char* kProfNames[6] = {"phi_eval", "density", "hs", "backward", "finish", "operands"};

// Runs one launch, bracketed by events when profiling is on.
template <typename F>
void timed(aims_grid* g, int kind, double work, const char* what, F&& launch,
           hipStream_t on = nullptr) {
  if (!g->profiling) {
    hipchk(launch(), what);
    return;
  }
  if (!on) on = g->stream;
  aims_grid::ProfRec r{kind, nullptr, nullptr, work};
  hipchk(hipEventCreate(&r.a), "event");
  hipchk(hipEventCreate(&r.b), "event");
  hipchk(hipEventRecord(r.a, on), "event");
  hipchk(launch(), what);
  hipchk(hipEventRecord(r.b, on), "event");
  g->prof_pending.push_back(r);
}

// The groups of one pass, in order on the handle's stream: each group's basis evaluation into
// the slab pair, then the group's tiles (every tile-shape run of the group).
// phi(gi, slab1, slab2, stream) and tiles(gi, slab1, slab2, stream) launch one group.
template <typename Phi, typename Tiles>
void run_groups(aims_grid* g, size_t ngroups, Phi&& phi, Tiles&& tiles) {
  for (size_t gi = 0; gi < ngroups; ++gi) {
    phi(gi, g->d_slab1, g->d_slab2, g->stream);
    tiles(gi, g->d_slab1, g->d_slab2, g->stream);
  }
}

void prof_collect(aims_grid* g) {
  if (g->prof_pending.empty()) return;
  hipchk(hipStreamSynchronize(g->stream), "profile sync");
  for (auto& r : g->prof_pending) {
    float ms = 0.f;
    hipchk(hipEventElapsedTime(&ms, r.a, r.b), "elapsed");
    g->prof_count[r.kind] += 1;
    g->prof_ms[r.kind] += ms;
    g->prof_work[r.kind] += r.work;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g->prof_pending.clear();
}

// Counters of the persistent tile launches of one call: all of them are cleared by one small
// kernel at the start of the call (no memset node, so the call may be captured into a graph),
// then each tiled launch takes the next 8.
struct QueueSeq {
  int* base = nullptr;
  size_t k = 0, cap = 0;
  QueueSeq(aims_grid* g, const ItemList& L, aims_precision prec, bool grid_only = false) {
    if (grid_only || !g->persistent[prec]) return;
    size_t launches = 0;
    for (const auto& r : L.runs) launches += r.size();
    if (8 * launches > g->queue_cap) fail(AIMS_ERR_ARG, "work counters not allocated");
    base = g->d_queue;
    cap = 8 * launches;
    hipchk(launch_zero_int(base, (int)cap, g->stream), "clear work counters");
  }
  Queue next() {
    Queue q;
    if (!base) return q;
    if (k + 8 > cap) fail(AIMS_ERR_ARG, "work counter overflow");
    q.counters = base + k;
    k += 8;
    return q;
  }
};

// Density update with basis values of precision T (double / float) on the MFMA type of T,
// or, with bf16x3, FP32 basis values split into bf16 hi/lo pairs.
//
// The allocation-free form (noalloc) runs the same kernels on the batch set grouped for the
// static scratch, with its slabs in that scratch, grid launches (no work counters) and no
// profiling events.
template <typename T>
void run_density(aims_grid* g, aims_precision prec, const T* P, const double* v, double* n_out,
                 double* sums_out, bool noalloc = false) {
  hipStream_t st = g->stream;
  BatchSet& bs = noalloc ? g->dens_na : g->dens;
  const int pblocks = noalloc ? kNoAllocPblocks : g->d_pblocks[prec];
  const ItemList* Lp = nullptr;
  if (noalloc) {
    for (auto& l : bs.lists)
      if (l->key == density_key(pblocks, nullptr)) Lp = l.get();
    if (!Lp) fail(AIMS_ERR_ARG, "allocation-free work list missing");
  } else {
    Lp = &tile_list(g, bs, dens_key_of(g, prec));
  }
  const ItemList& L = *Lp;
  void* na_slab1 = g->na_scratch;
  void* na_slab2 = (void*)((unsigned char*)g->na_scratch + kNoAllocScratchBytes / 2);
  auto timed = [&](int kind, double work, const char* what, auto&& launch, hipStream_t on) {
    if (noalloc) hipchk(launch(), what);
    else ::timed(g, kind, work, what, launch, on);
  };
  hipchk(launch_fill(g->d_n_sorted, (size_t)g->n_points, 0.0, st), "fill n");
  hipchk(launch_fill(g->d_et_batch, bs.batches.size(), 0.0, st), "fill E_T");
  QueueSeq qs(g, L, noalloc ? AIMS_FP64 : prec, noalloc);
  auto phi = [&](size_t gi, void* slab1, void* slab2, hipStream_t on) {
    const auto& gr = bs.groups[gi];
    const int nbt = gr.b1 - gr.b0;
    timed(kProfPhi, 0.0, "phi_eval", [&] {
      if (prec == AIMS_BF16X3)
        return launch_phi_eval_bf16(bs.dv, gr.b0, nbt, kModeDensity, nullptr, slab1, slab2, on);
      return launch_phi_eval<T>(bs.dv, gr.b0, nbt, kModeDensity, nullptr, (T*)slab1, (T*)slab2, on);
    }, on);
  };
  auto tiles = [&](size_t gi, void* slab1, void* slab2, hipStream_t on) {
    const auto& gr = bs.groups[gi];
    for (size_t r = 0; r < L.runs[gi].size(); ++r) {
      const auto& run = L.runs[gi][r];
      const double work = r + 1 == L.runs[gi].size() ? gr.flops : 0.0;   // credited once per group
      const int nit = (int)(run.i1 - run.i0);
      if (prec == AIMS_BF16X3) {
        timed(kProfDensity, work, "density", [&] {
          return launch_density_bf16(bs.dv, run.nbn, L.d_items + run.i0, nit, (const float*)P,
                                     slab1, slab2, g->d_n_sorted, g->d_et_batch, on,
                                     nullptr, qs.next());
        }, on);
      } else {
        timed(kProfDensity, work, "density", [&] {
          return launch_density<T>(bs.dv, run.nbn, L.d_items + run.i0, nit, P, (const T*)slab1,
                                   (const T*)slab2, g->d_n_sorted, g->d_et_batch, on, nullptr,
                                   qs.next());
        }, on);
      }
    }
  };
  if (noalloc) {
    for (size_t gi = 0; gi < bs.groups.size(); ++gi) {
      phi(gi, na_slab1, na_slab2, st);
      tiles(gi, na_slab1, na_slab2, st);
    }
  } else {
    run_groups(g, bs.groups.size(), phi, tiles);
  }
  timed(kProfFinish, 0.0, "density_finish", [&] {
    return launch_density_finish(bs.dv, g->d_n_sorted, v, n_out, g->d_part, g->nblk_finish,
                                 g->d_et_batch, sums_out, st);
  }, st);
}

template <typename T>
void run_hs(aims_grid* g, aims_precision prec, int mode, const double* v, double* out,
            const double* u = nullptr) {
  hipStream_t st = g->stream;
  BatchSet& bs = hset(g, g->h_merge[prec], g->h_ratio[prec]);
  const ItemList& L = tile_list(g, bs, h_key_of(g, prec));
  hipchk(launch_fill(out, (size_t)g->mat_total, 0.0, st), "fill H");
  QueueSeq qs(g, L, prec);
  auto phi = [&](size_t gi, void* s1, void* s2, hipStream_t on) {
    const auto& gr = bs.groups[gi];
    const int nbt = gr.b1 - gr.b0;
    timed(g, kProfPhi, 0.0, "phi_eval", [&] {
      if (prec == AIMS_BF16X3) return launch_phi_eval_bf16(bs.dv, gr.b0, nbt, mode, v, s1, s2, on);
      return launch_phi_eval<T>(bs.dv, gr.b0, nbt, mode, v, (T*)s1, (T*)s2, on);
    }, on);
    if (u)
      timed(g, kProfPhi, 0.0, "vector term", [&] {
        return launch_vector_term<T>(bs.dv, gr.b0, nbt, u, (T*)s2, on);
      }, on);
  };
  auto tiles = [&](size_t gi, void* s1, void* s2, hipStream_t on) {
    const auto& gr = bs.groups[gi];
    for (const auto& run : L.runs[gi]) {
      const int nit = (int)(run.i1 - run.i0);
      timed(g, kProfHS, gr.flops, "hs", [&] {
        if (prec == AIMS_BF16X3)
          return launch_hs_bf16(bs.dv, L.d_items + run.i0, nit, s1, s2, out, on, qs.next());
        return launch_hs<T>(bs.dv, L.d_items + run.i0, nit, (const T*)s1, (const T*)s2, out, on,
                            qs.next(), run.nbn ? 32 : 64);
      }, on);
    }
  };
  run_groups(g, bs.groups.size(), phi, tiles);
}

// ---- sliced integer form ------------------------------------------------------------------
// Buffers of the int8 form, taken on first use (and before a step graph is captured).
void prepare_i8(aims_grid* g, BatchSet* hbs) {
  if (!g->d_P8) {
    g->d_P8 = (uint64_t*)g->alloc(std::max<int64_t>(1, g->mat_total) * sizeof(uint64_t));
    g->d_eP = (int32_t*)g->alloc(std::max<int64_t>(1, g->nb_total) * sizeof(int32_t));
    g->d_pexp = (int32_t*)g->alloc(2 * std::max<int64_t>(1, g->n_points) * sizeof(int32_t));
  }
  if (hbs && !hbs->d_colexp)
    hbs->d_colexp = (int32_t*)g->alloc(2 * std::max<size_t>(1, hbs->batch_cols.size()) * sizeof(int32_t));
}

// Largest basis slab row length (density: ldp) or basis count (H / S) of a group's batches: the
// basis evaluation keeps one LDS slot pair per point or per function (64 KiB at most).
int group_slots(const BatchSet& bs, const BatchSet::Group& gr, bool per_point) {
  int m = 0;
  for (int b = gr.b0; b < gr.b1; ++b) m = std::max(m, per_point ? bs.batches[b].ldp : bs.batches[b].n_b);
  if (m > 4096) fail(AIMS_ERR_UNSUPPORTED, "AIMS_INT8X7: a batch of %d functions (at most 4096)", m);
  return m;
}

void run_density_i8(aims_grid* g, const double* P, const double* v, double* n_out, double* sums_out) {
  hipStream_t st = g->stream;
  BatchSet& bs = g->dens;
  prepare_i8(g, nullptr);
  const ItemList& L = tile_list(g, bs, dens_key_of(g, AIMS_INT8X7));
  int32_t* ex1 = g->d_pexp;
  int32_t* ex2 = g->d_pexp + g->n_points;
  timed(g, kProfOperands, 0.0, "slice P", [&] {
    return launch_slice_p(bs.dv, P, g->d_P8, g->d_eP, g->nb_total, st);
  });
  hipchk(launch_fill(g->d_n_sorted, (size_t)g->n_points, 0.0, st), "fill n");
  hipchk(launch_fill(g->d_et_batch, bs.batches.size(), 0.0, st), "fill E_T");
  QueueSeq qs(g, L, AIMS_INT8X7);
  auto phi = [&](size_t gi, void* s1, void* s2, hipStream_t on) {
    const auto& gr = bs.groups[gi];
    const int slots = group_slots(bs, gr, true);
    timed(g, kProfPhi, 0.0, "phi_eval", [&] {
      return launch_phi_eval_i8(bs.dv, gr.b0, gr.b1 - gr.b0, kModeDensity, nullptr, (uint64_t*)s1,
                                (uint64_t*)s2, ex1, ex2, slots, on);
    }, on);
  };
  auto tiles = [&](size_t gi, void* s1, void* s2, hipStream_t on) {
    const auto& gr = bs.groups[gi];
    for (size_t r = 0; r < L.runs[gi].size(); ++r) {
      const auto& run = L.runs[gi][r];
      if (run.nbn != 2) fail(AIMS_ERR_ARG, "AIMS_INT8X7 density tiles span 64 points");
      const double work = r + 1 == L.runs[gi].size() ? gr.flops : 0.0;
      timed(g, kProfDensity, work, "density", [&] {
        return launch_density_i8(bs.dv, L.d_items + run.i0, (int)(run.i1 - run.i0), g->d_P8, g->d_eP,
                                 (const uint64_t*)s1, (const uint64_t*)s2, ex1, ex2, g->d_n_sorted,
                                 g->d_et_batch, on, qs.next());
      }, on);
    }
  };
  run_groups(g, bs.groups.size(), phi, tiles);
  timed(g, kProfFinish, 0.0, "density_finish", [&] {
    return launch_density_finish(bs.dv, g->d_n_sorted, v, n_out, g->d_part, g->nblk_finish,
                                 g->d_et_batch, sums_out, st);
  });
}

void run_hs_i8(aims_grid* g, int mode, const double* v, double* out) {
  hipStream_t st = g->stream;
  BatchSet& bs = hset(g, g->h_merge[AIMS_INT8X7], g->h_ratio[AIMS_INT8X7]);
  prepare_i8(g, &bs);
  const ItemList& L = tile_list(g, bs, h_key(0));
  int32_t* ex1 = bs.d_colexp;
  int32_t* ex2 = bs.d_colexp + bs.batch_cols.size();
  hipchk(launch_fill(out, (size_t)g->mat_total, 0.0, st), "fill H");
  QueueSeq qs(g, L, AIMS_INT8X7);
  auto phi = [&](size_t gi, void* s1, void* s2, hipStream_t on) {
    const auto& gr = bs.groups[gi];
    const int slots = group_slots(bs, gr, false);
    timed(g, kProfPhi, 0.0, "phi_eval", [&] {
      return launch_phi_eval_i8(bs.dv, gr.b0, gr.b1 - gr.b0, mode, v, (uint64_t*)s1, (uint64_t*)s2,
                                ex1, ex2, slots, on);
    }, on);
  };
  auto tiles = [&](size_t gi, void* s1, void* s2, hipStream_t on) {
    const auto& gr = bs.groups[gi];
    for (const auto& run : L.runs[gi])
      timed(g, kProfHS, gr.flops, "hs", [&] {
        return launch_hs_i8(bs.dv, L.d_items + run.i0, (int)(run.i1 - run.i0), (const uint64_t*)s1,
                            (const uint64_t*)s2, ex1, ex2, out, on, qs.next());
      }, on);
  };
  run_groups(g, bs.groups.size(), phi, tiles);
}

// One precision-dispatched density update (P converted to FP32 for the mixed forms).
void density_call(aims_grid* g, aims_precision prec, const double* P, const double* v, double* n_out,
                  double* sums_out, bool noalloc = false) {
  if (prec == AIMS_INT8X7) {
    if (noalloc) fail(AIMS_ERR_UNSUPPORTED, "the allocation-free update takes AIMS_FP64, AIMS_FP32 or AIMS_BF16X3");
    run_density_i8(g, P, v, n_out, sums_out);
  } else if (prec == AIMS_FP64) {
    run_density<double>(g, prec, P, v, n_out, sums_out, noalloc);
  } else {
    hipchk(launch_convert_f32(P, g->d_P32, (size_t)g->mat_total, g->stream), "convert P");
    run_density<float>(g, prec, g->d_P32, v, n_out, sums_out, noalloc);
  }
}

void hs_call(aims_grid* g, aims_precision prec, int mode, const double* v, double* out,
             const double* u = nullptr) {
  if (prec == AIMS_INT8X7) {
    if (u) fail(AIMS_ERR_UNSUPPORTED, "AIMS_INT8X7 has no gradient term of H");
    run_hs_i8(g, mode, v, out);
  } else if (prec == AIMS_FP64) {
    run_hs<double>(g, prec, mode, v, out, u);
  } else {
    run_hs<float>(g, prec, mode, v, out, u);
  }
}

// A roctx range around each C-ABI call, so that traces (rocprofv3 --marker-trace) show which
// call issued which kernels.
struct CallRange {
  explicit CallRange(const char* name) { roctxRangePush(name); }
  ~CallRange() { roctxRangePop(); }
};

template <typename F>
aims_status guarded(const char* name, aims_grid* g, F&& f) {
  CallRange range(name);
  try {
    if (!g) fail(AIMS_ERR_ARG, "null handle");
    hipchk(hipSetDevice(g->device), "hipSetDevice");
    f();
    return AIMS_OK;
  } catch (const Fail& e) {
    if (g) g->err = e.msg;
    else g_setup_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    if (g) g->err = "host allocation failed";
    return AIMS_ERR_OOM;
  }
}

// Tables of the wave-per-point force kernel (setup positions, current partition parameters):
// 1 / (a |R_b - R_c|) per system, and runs of consecutive batches of one system holding about
// the same number of points, about kForceRanges of them in all.
constexpr int kForceRanges = 4096;
constexpr int kForceWaveMaxAtoms = 512;

void build_force_tables(aims_grid* g, int max_na) {
  int k = 1;
  while (64 * k < max_na) k *= 2;
  std::vector<int64_t> pair_off(g->n_sys);
  int64_t tot = 0;
  for (int s = 0; s < g->n_sys; ++s) {
    const int64_t na = g->sys_atom_range[2 * s + 1] - g->sys_atom_range[2 * s];
    pair_off[s] = tot;
    tot += na * na;
  }
  std::vector<double> inv(std::max<int64_t>(1, tot), 0.0);
  for (int s = 0; s < g->n_sys; ++s) {
    const int a0 = (int)g->sys_atom_range[2 * s], na = (int)(g->sys_atom_range[2 * s + 1] - a0);
    const double a = g->sys_model[2 * s + 1];
    const double* X = g->atom_xyz0.data() + 3 * (size_t)a0;
    for (int b = 0; b < na; ++b)
      for (int c = 0; c < na; ++c) {
        if (b == c) continue;
        const double dx = X[3 * b] - X[3 * c], dy = X[3 * b + 1] - X[3 * c + 1], dz = X[3 * b + 2] - X[3 * c + 2];
        const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
        if (!(r > 0.0)) fail(AIMS_ERR_ARG, "system %d: atoms %d and %d coincide", s, b, c);
        inv[pair_off[s] + (int64_t)b * na + c] = 1.0 / (a * r);
      }
  }
  const BatchSet& bs = g->dens;
  const int64_t nb_all = (int64_t)bs.batches.size();
  std::vector<ForceRange> ranges;
  std::vector<int64_t> part_off(g->n_sys, 0);
  std::vector<int32_t> nrange(g->n_sys, 0);
  int64_t cursor = 0;
  for (int s = 0; s < g->n_sys; ++s) {
    const int na = (int)(g->sys_atom_range[2 * s + 1] - g->sys_atom_range[2 * s]);
    const int64_t B0 = bs.sys_batch_range[2 * s], B1 = bs.sys_batch_range[2 * s + 1];
    part_off[s] = cursor;
    if (B1 <= B0) continue;
    int64_t npts = 0;
    for (int64_t b = B0; b < B1; ++b) npts += bs.batches[b].n_p;
    const int64_t want = std::max<int64_t>(1, std::min<int64_t>(B1 - B0, (kForceRanges * (B1 - B0) + nb_all - 1) / nb_all));
    const double per = (double)npts / (double)want;
    int64_t b = B0, acc = 0;
    for (int64_t r = 0; r < want && b < B1; ++r) {
      const int64_t start = b;
      const double goal = per * (double)(r + 1);
      while (b < B1 && (b == start || (double)(acc + bs.batches[b].n_p) <= goal + 0.5 * per)) acc += bs.batches[b++].n_p;
      if (r == want - 1) while (b < B1) acc += bs.batches[b++].n_p;
      ranges.push_back(ForceRange{(int32_t)start, (int32_t)b, s, 0, cursor});
      cursor += 3 * (int64_t)na;
      ++nrange[s];
    }
  }
  auto drop = [&](auto*& ptr) {
    if (ptr) g->release(ptr);
    ptr = nullptr;
  };
  drop(g->d_franges);
  drop(g->d_inv_aR);
  drop(g->d_pair_off);
  drop(g->d_fpart);
  drop(g->d_fpart_off);
  drop(g->d_fnrange);
  g->d_inv_aR = g->upload(inv);
  g->d_pair_off = g->upload(pair_off);
  if (ranges.empty()) ranges.push_back(ForceRange{0, 0, 0, 0, 0});     // a valid (unused) entry
  g->d_franges = g->upload(ranges);
  g->gf_nranges = (int)(ranges.size() == 1 && ranges[0].b1 == 0 ? 0 : ranges.size());
  g->d_fpart = (double*)g->alloc(std::max<int64_t>(1, cursor) * sizeof(double));
  g->d_fpart_off = g->upload(part_off);
  g->d_fnrange = g->upload(nrange);
  g->gf_k = k;
  g->gf_ready = true;
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's iteration on P_n from the three-term
// recurrence, w = 2 / ((1 - x^2) P_n'(x)^2)
std::vector<double> gauss_legendre(int n) {
  std::vector<double> out(2 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    out[n - 1 - i] = x;                                  // ascending
    out[n + (n - 1 - i)] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return out;
}

void build_hartree(aims_grid* g) {
  const int L = g->hartree_lmax, nlm = (L + 1) * (L + 1);
  int K_max = 0;
  for (int k : g->h_K) K_max = std::max(K_max, k);
  // shells: every (atom, node), points grouped by (atom, node) in batch-order indices
  std::vector<HartreeShell> shells;
  std::vector<int32_t> count((size_t)g->n_atoms * K_max, 0);
  for (int64_t i = 0; i < g->n_points; ++i) ++count[(size_t)g->h_owner[i] * K_max + g->h_node[i]];
  std::vector<int32_t> start(count.size() + 1, 0);
  for (size_t c = 0; c < count.size(); ++c) start[c + 1] = start[c] + count[c];
  std::vector<int32_t> pts_sorted(std::max<int64_t>(1, g->n_points));
  std::vector<int32_t> fill(start.begin(), start.end() - 1);
  for (int64_t i = 0; i < g->n_points; ++i)
    pts_sorted[fill[(size_t)g->h_owner[i] * K_max + g->h_node[i]]++] = (int32_t)i;
  std::vector<HartreeSys> hs(g->n_sys);
  std::vector<double> cp, den;
  std::vector<int32_t> natoms(g->n_sys);
  // edge node per atom: one node outwards (towards node 0) of the outermost node with a point
  std::vector<int32_t> edge(g->n_atoms, 0);
  std::vector<double> r_edge(g->n_atoms, 0.0);
  for (int s = 0; s < g->n_sys; ++s) {
    const int K = g->h_K[s];
    const double rm = g->h_rmap[s];
    hs[s] = HartreeSys{K, K_max, (int32_t)cp.size(), 0, rm};
    // Thomas factors of M_{i-1} + 4 M_i + M_{i+1} = rhs_i (i = 1..K-2), natural ends
    std::vector<double> c(K, 0.0), d(K, 1.0);
    for (int i = 1; i <= K - 2; ++i) {
      d[i] = i == 1 ? 4.0 : 4.0 - c[i - 1];
      c[i] = 1.0 / d[i];
    }
    cp.insert(cp.end(), c.begin(), c.end());
    den.insert(den.end(), d.begin(), d.end());
    const int a0 = (int)g->sys_atom_range[2 * s], a1 = (int)g->sys_atom_range[2 * s + 1];
    natoms[s] = a1 - a0;
    for (int a = a0; a < a1; ++a) {
      int ko = -1;
      for (int k = 0; k < K && ko < 0; ++k)
        if (count[(size_t)a * K_max + k] > 0) ko = k;
      edge[a] = ko > 0 ? ko - 1 : 0;
      const double te = (double)(edge[a] + 1) * M_PI / (double)(K + 1), xe = std::cos(te);
      r_edge[a] = rm * (1.0 + xe) / (1.0 - xe);
    }
    for (int a = a0; a < a1; ++a)
      for (int k = 0; k < K; ++k) {
        // Becke radial weight with r^2: W = pi/(K+1) sin t 2 r_m/(1 - cos t)^2 r^2
        const double t = (double)(k + 1) * M_PI / (double)(K + 1), x = std::cos(t);
        const double r = rm * (1.0 + x) / (1.0 - x);
        const double W = M_PI / (double)(K + 1) * std::sin(t) * 2.0 * rm / ((1.0 - x) * (1.0 - x)) * r * r;
        const size_t cidx = (size_t)a * K_max + k;
        shells.push_back(HartreeShell{a, start[cidx], start[cidx + 1], (int32_t)cidx, 1.0 / W});
      }
  }
  HartreeDev& hd = g->hd;
  auto drop = [&](auto* p) {
    if (p) g->release((void*)p);
  };
  drop(hd.shells);
  drop(hd.shell_pts);
  drop(hd.sys);
  drop(hd.sys_natoms);
  drop(hd.edge);
  drop(hd.r_edge);
  drop(hd.cp);
  drop(hd.den);
  drop(hd.gl);
  drop(hd.rho);
  drop(hd.Mr);
  drop(hd.V);
  drop(hd.MV);
  drop(hd.q);
  drop(hd.Vc);
  drop(hd.part);
  hd = HartreeDev{};
  hd.l_max = L;
  hd.n_atoms = g->n_atoms;
  hd.n_shells = (int)shells.size();
  hd.shells = g->upload(shells);
  hd.shell_pts = g->upload(pts_sorted);
  hd.sys = g->upload(hs);
  hd.sys_natoms = g->upload(natoms);
  hd.edge = g->upload(edge);
  hd.r_edge = g->upload(r_edge);
  hd.cp = g->upload(cp);
  hd.den = g->upload(den);
  hd.gl = g->upload(gauss_legendre(kGauss));
  const size_t nodes = std::max<size_t>(1, (size_t)g->n_atoms * K_max * nlm);
  hd.rho = (double*)g->alloc(nodes * sizeof(double));
  hd.Mr = (double*)g->alloc(nodes * sizeof(double));
  hd.V = (double*)g->alloc(nodes * sizeof(double));
  hd.MV = (double*)g->alloc(nodes * sizeof(double));
  hd.q = (double*)g->alloc(std::max<size_t>(1, (size_t)g->n_atoms * nlm) * sizeof(double));
  hd.Vc = (double4*)g->alloc(nodes * sizeof(double4));
  hd.part = (double*)g->alloc((size_t)g->n_sys * kHartreeBlocks * sizeof(double));
  g->h_ready = true;
}

}  // namespace

// -------------------------------------------------------------------------------------------------
// C ABI
// -------------------------------------------------------------------------------------------------
extern "C" {

aims_status aims_grid_setup_many(const aims_system* sys, int32_t n_sys, int device, void* hip_stream,
                                 aims_grid** out) {
  try {
    if (!out) fail(AIMS_ERR_ARG, "out is NULL");
    *out = nullptr;
    *out = build(sys, n_sys, device, hip_stream);
    return AIMS_OK;
  } catch (const Fail& e) {
    g_setup_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    g_setup_error = "host allocation failed";
    return AIMS_ERR_OOM;
  }
}

aims_status aims_grid_setup(const aims_system* sys, int device, void* hip_stream, aims_grid** out) {
  return aims_grid_setup_many(sys, 1, device, hip_stream, out);
}

aims_status aims_update_density(aims_grid* g, aims_precision prec, const double* atom_xyz,
                                const double* P, const double* v_or_null, double* n_out,
                                double* sums_out) {
  return guarded(__func__, g, [&] {
    check_prec(prec);
    require_device(P, "P", (size_t)g->mat_total * sizeof(double));
    require_device(n_out, "n_out", (size_t)g->n_points * sizeof(double));
    require_device(sums_out, "sums_out", 3 * (size_t)g->n_sys * sizeof(double));
    debug_check_symmetric(g, P, "P");
    if (v_or_null) require_device(v_or_null, "v", (size_t)g->n_points * sizeof(double));
    set_positions(g, atom_xyz);
    density_call(g, prec, P, v_or_null, n_out, sums_out);
    poison_outputs(g, n_out, (size_t)g->n_points);
    poison_outputs(g, sums_out, 3 * (size_t)g->n_sys);
  });
}

aims_status aims_update_density_noalloc(aims_grid* g, aims_precision prec, const double* P,
                                        const double* v_or_null, double* n_out, double* sums_out) {
  return guarded(__func__, g, [&] {
    check_prec(prec);
    require_device(P, "P", (size_t)g->mat_total * sizeof(double));
    require_device(n_out, "n_out", (size_t)g->n_points * sizeof(double));
    require_device(sums_out, "sums_out", 3 * (size_t)g->n_sys * sizeof(double));
    if (v_or_null) require_device(v_or_null, "v", (size_t)g->n_points * sizeof(double));
    debug_check_symmetric(g, P, "P");
    if (!g->na_error.empty()) fail(AIMS_ERR_UNSUPPORTED, "%s", g->na_error.c_str());
    set_positions(g, nullptr);
    density_call(g, prec, P, v_or_null, n_out, sums_out, true);
  });
}

aims_status aims_integrate_h(aims_grid* g, aims_precision prec, const double* atom_xyz, const double* v,
                             double* H, double* S_or_null) {
  return guarded(__func__, g, [&] {
    check_prec(prec);
    require_device(v, "v", (size_t)g->n_points * sizeof(double));
    require_device(H, "H", (size_t)g->mat_total * sizeof(double));
    if (S_or_null) require_device(S_or_null, "S", (size_t)g->mat_total * sizeof(double));
    set_positions(g, atom_xyz);
    hs_call(g, prec, kModeH, v, H);
    if (S_or_null) hs_call(g, prec, kModeS, v, S_or_null);
    poison_outputs(g, H, (size_t)g->mat_total);
    poison_outputs(g, S_or_null, (size_t)g->mat_total);
  });
}

aims_status aims_integrate_h_gga(aims_grid* g, aims_precision prec, const double* v,
                                 const double* u, double* H) {
  return guarded(__func__, g, [&] {
    check_prec(prec);
    if (prec == AIMS_BF16X3 || prec == AIMS_INT8X7)
      fail(AIMS_ERR_UNSUPPORTED, "the gradient term supports AIMS_FP64 and AIMS_FP32");
    require_device(v, "v", (size_t)g->n_points * sizeof(double));
    require_device(u, "u", 3 * (size_t)g->n_points * sizeof(double));
    require_device(H, "H", (size_t)g->mat_total * sizeof(double));
    set_positions(g, nullptr);
    if (g->moved) fail(AIMS_ERR_ARG, "the gradient term is integrated at the setup positions");
    hs_call(g, prec, kModeH, v, H, u);
  });
}

aims_status aims_integrate_h_backward(aims_grid* g, aims_precision prec, const double* atom_xyz,
                                      const double* P, const double* v, const double* gE,
                                      double* dE_dP_or_null, double* dE_dv_or_null,
                                      double* dE_dR_or_null) {
  return guarded(__func__, g, [&] {
    check_prec(prec);
    forward_only(prec, "the backward");
    require_device(P, "P", (size_t)g->mat_total * sizeof(double));
    require_device(v, "v", (size_t)g->n_points * sizeof(double));
    require_device(gE, "gE", sizeof(double));
    if (dE_dP_or_null) require_device(dE_dP_or_null, "dE_dP", (size_t)g->mat_total * sizeof(double));
    if (dE_dv_or_null) require_device(dE_dv_or_null, "dE_dv", (size_t)g->n_points * sizeof(double));
    debug_check_symmetric(g, P, "P");
    if (dE_dR_or_null) require_device(dE_dR_or_null, "dE_dR", 3 * (size_t)g->n_atoms * sizeof(double));
    set_positions(g, atom_xyz);
    hipStream_t st = g->stream;
    if (!g->d_ntmp) {
      g->d_ntmp = (double*)g->alloc(std::max<int64_t>(1, g->n_points) * sizeof(double));
      g->d_sums_tmp = (double*)g->alloc(3 * (size_t)g->n_sys * sizeof(double));
    }
    // dE/dP = gE H
    if (dE_dP_or_null) {
      hs_call(g, prec, kModeH, v, dE_dP_or_null);
      hipchk(launch_scale(dE_dP_or_null, dE_dP_or_null, (size_t)g->mat_total, gE, st), "scale dE/dP");
    }
    if (!dE_dv_or_null && !dE_dR_or_null) {
      poison_outputs(g, dE_dP_or_null, (size_t)g->mat_total);
      return;
    }
    if (!dE_dR_or_null) {
      // n (for dE/dv) from a plain density pass
      density_call(g, prec, P, v, g->d_ntmp, g->d_sums_tmp);
      hipchk(launch_dv(g->dens.dv, dE_dv_or_null, g->d_n_sorted, g->n_points, gE, st), "dE/dv");
      poison_outputs(g, dE_dP_or_null, (size_t)g->mat_total);
      poison_outputs(g, dE_dv_or_null, (size_t)g->n_points);
      return;
    }
    // dE/dR: X = Phi P_b (whose pass also forms n, for dE/dv) and Y = (T Phi) P_b per batch,
    // then the Pulay reduction
    BatchSet& bs = g->dens;
    if (g->slab_cap34 < bs.slab_elems) {
      if (g->d_slab3) g->release(g->d_slab3);
      if (g->d_slab4) g->release(g->d_slab4);
      g->d_slab3 = g->d_slab4 = nullptr;
      g->slab_cap34 = 0;
      g->d_slab3 = g->alloc(bs.slab_elems * sizeof(double));
      g->d_slab4 = g->alloc(bs.slab_elems * sizeof(double));
      g->slab_cap34 = bs.slab_elems;
    }
    const bool mixed = prec != AIMS_FP64;
    if (mixed) hipchk(launch_convert_f32(P, g->d_P32, (size_t)g->mat_total, st), "convert P");
    hipchk(launch_fill(g->d_n_sorted, (size_t)g->n_points, 0.0, st), "fill n");
    hipchk(launch_fill(g->d_et_batch, bs.batches.size(), 0.0, st), "fill E_T");
    hipchk(launch_fill(dE_dR_or_null, 3 * (size_t)g->n_atoms, 0.0, st), "fill dE/dR");
    const ItemList& L = tile_list(g, bs, dens_key_of(g, prec));
    for (size_t gi = 0; gi < bs.groups.size(); ++gi) {
      const auto& gr = bs.groups[gi];
      const int nbt = gr.b1 - gr.b0;
      if (!mixed) {
        double *s1 = (double*)g->d_slab1, *s2 = (double*)g->d_slab2;
        double *s3 = (double*)g->d_slab3, *s4 = (double*)g->d_slab4;
        timed(g, kProfPhi, 0.0, "phi_eval", [&] {
          return launch_phi_eval<double>(bs.dv, gr.b0, nbt, kModeDensity, nullptr, s1, s2, st);
        });
        for (const auto& run : L.runs[gi]) {
          const int nit = (int)(run.i1 - run.i0);
          timed(g, kProfBackward, gr.flops / L.runs[gi].size(), "X", [&] {
            return launch_density<double>(bs.dv, run.nbn, L.d_items + run.i0, nit, P, s1, s2,
                                          g->d_n_sorted, g->d_et_batch, st, s3);
          });
          timed(g, kProfBackward, gr.flops / L.runs[gi].size(), "Y", [&] {
            return launch_density<double>(bs.dv, run.nbn, L.d_items + run.i0, nit, P, s2, s2, nullptr,
                                          nullptr, st, s4);
          });
        }
        timed(g, kProfBackward, 0.0, "pulay", [&] {
          return launch_pulay<double>(bs.dv, gr.b0, nbt, v, s3, s4, gE, dE_dR_or_null, st);
        });
      } else {
        float *s3 = (float*)g->d_slab3, *s4 = (float*)g->d_slab4;
        if (prec == AIMS_BF16X3) {
          timed(g, kProfPhi, 0.0, "phi_eval", [&] {
            return launch_phi_eval_bf16(bs.dv, gr.b0, nbt, kModeDensity, nullptr, g->d_slab1, g->d_slab2, st);
          });
        } else {
          timed(g, kProfPhi, 0.0, "phi_eval", [&] {
            return launch_phi_eval<float>(bs.dv, gr.b0, nbt, kModeDensity, nullptr, (float*)g->d_slab1,
                                          (float*)g->d_slab2, st);
          });
        }
        for (const auto& run : L.runs[gi]) {
          const int nit = (int)(run.i1 - run.i0);
          for (int which = 0; which < 2; ++which) {
            const void* src = which == 0 ? g->d_slab1 : g->d_slab2;
            float* dst = which == 0 ? s3 : s4;
            double* nout = which == 0 ? g->d_n_sorted : nullptr;
            double* eout = which == 0 ? g->d_et_batch : nullptr;
            timed(g, kProfBackward, gr.flops / L.runs[gi].size(), "XY", [&] {
              if (prec == AIMS_BF16X3)
                return launch_density_bf16(bs.dv, run.nbn, L.d_items + run.i0, nit, g->d_P32, src,
                                           g->d_slab2, nout, eout, st, dst);
              return launch_density<float>(bs.dv, run.nbn, L.d_items + run.i0, nit, g->d_P32,
                                           (const float*)src, (const float*)g->d_slab2, nout, eout,
                                           st, dst);
            });
          }
        }
        timed(g, kProfBackward, 0.0, "pulay", [&] {
          return launch_pulay<float>(bs.dv, gr.b0, nbt, v, s3, s4, gE, dE_dR_or_null, st);
        });
      }
    }
    if (dE_dv_or_null)
      hipchk(launch_dv(g->dens.dv, dE_dv_or_null, g->d_n_sorted, g->n_points, gE, st), "dE/dv");
    poison_outputs(g, dE_dP_or_null, (size_t)g->mat_total);
    poison_outputs(g, dE_dv_or_null, (size_t)g->n_points);
    poison_outputs(g, dE_dR_or_null, 3 * (size_t)g->n_atoms);
  });
}

aims_status aims_grid_set_moving(aims_grid* g, int32_t sys, const aims_moving_grid* m) {
  return guarded(__func__, g, [&] {
    if (!m) fail(AIMS_ERR_ARG, "null moving-grid description");
    if (sys < 0 || sys >= g->n_sys) fail(AIMS_ERR_ARG, "system %d out of range", sys);
    if (!(m->nuc_sigma > 0.0) || !std::isfinite(m->nuc_sigma)) fail(AIMS_ERR_ARG, "nuc_sigma must be > 0");
    if (!(m->partition_a > 0.0 && m->partition_a < 1.0)) fail(AIMS_ERR_ARG, "partition_a must be in (0, 1)");
    const int64_t p0 = g->sys_pt_range[2 * sys], p1 = g->sys_pt_range[2 * sys + 1];
    const int a0 = (int)g->sys_atom_range[2 * sys], a1 = (int)g->sys_atom_range[2 * sys + 1];
    if (p1 > p0 && (!m->pt_owner || !m->pt_wgrid)) fail(AIMS_ERR_ARG, "null point arrays");
    if (!m->atom_Z) fail(AIMS_ERR_ARG, "null atom_Z");
    if (!finite_all(m->atom_Z, (size_t)(a1 - a0))) fail(AIMS_ERR_ARG, "non-finite atom_Z");
    if (p1 > p0 && !finite_all(m->pt_wgrid, (size_t)(p1 - p0))) fail(AIMS_ERR_ARG, "non-finite pt_wgrid");
    for (int64_t i = 0; i < p1 - p0; ++i)
      if (m->pt_owner[i] < 0 || m->pt_owner[i] >= a1 - a0)
        fail(AIMS_ERR_ARG, "pt_owner[%lld] = %d out of range", (long long)i, m->pt_owner[i]);
    const size_t n = (size_t)g->n_points;
    if (g->moving.empty()) {
      g->moving.assign(g->n_sys, 0);
      g->sys_model.assign(2 * (size_t)g->n_sys, 0.0);
      g->owner_host.assign(n, 0);
      g->wgrid_host.assign(n, 0.0);
      g->Z_host.assign(g->n_atoms, 0.0);
      g->pt_sys_host.assign(n, 0);
      for (int k = 0; k < g->n_sys; ++k)
        for (int64_t i = g->sys_pt_range[2 * k]; i < g->sys_pt_range[2 * k + 1]; ++i) g->pt_sys_host[i] = k;
      g->d_owner = (int32_t*)g->alloc(std::max<size_t>(1, n) * sizeof(int32_t));
      g->d_wgrid = (double*)g->alloc(std::max<size_t>(1, n) * sizeof(double));
      g->d_Z = (double*)g->alloc(std::max(1, g->n_atoms) * sizeof(double));
      g->d_sys_model = (double*)g->alloc(2 * (size_t)g->n_sys * sizeof(double));
      g->d_pt_sys = g->upload(g->pt_sys_host);
      std::vector<int32_t> natoms(g->n_sys);
      for (int k = 0; k < g->n_sys; ++k) natoms[k] = (int32_t)(g->sys_atom_range[2 * k + 1] - g->sys_atom_range[2 * k]);
      g->d_sys_natoms = g->upload(natoms);
      g->d_vmodel = (double*)g->alloc(std::max<size_t>(1, n) * sizeof(double));
      g->d_dsorted = (double*)g->alloc(std::max<size_t>(1, n) * sizeof(double));
      g->d_gpt = (double*)g->alloc(3 * std::max<size_t>(1, n) * sizeof(double));
    }
    for (int64_t i = p0; i < p1; ++i) {
      const int64_t q = g->perm_host[i] - p0;     // caller index within the system
      g->owner_host[i] = a0 + m->pt_owner[q];
      g->wgrid_host[i] = m->pt_wgrid[q];
    }
    for (int a = a0; a < a1; ++a) g->Z_host[a] = m->atom_Z[a - a0];
    g->sys_model[2 * sys] = m->nuc_sigma;
    g->sys_model[2 * sys + 1] = m->partition_a;
    g->moving[sys] = 1;
    g->gf_ready = false;
    hipchk(hipMemcpy(g->d_owner, g->owner_host.data(), n * sizeof(int32_t), hipMemcpyHostToDevice), "upload");
    hipchk(hipMemcpy(g->d_wgrid, g->wgrid_host.data(), n * sizeof(double), hipMemcpyHostToDevice), "upload");
    hipchk(hipMemcpy(g->d_Z, g->Z_host.data(), g->Z_host.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
    hipchk(hipMemcpy(g->d_sys_model, g->sys_model.data(), g->sys_model.size() * sizeof(double),
                     hipMemcpyHostToDevice), "upload");
  });
}

aims_status aims_total_forces(aims_grid* g, aims_precision prec, const double* P, const double* gE,
                              double* sums_out_or_null, double* dE_dR) {
  return guarded(__func__, g, [&] {
    check_prec(prec);
    if (prec == AIMS_BF16X3 || prec == AIMS_INT8X7)
      fail(AIMS_ERR_UNSUPPORTED, "total forces support AIMS_FP64 and AIMS_FP32");
    if (g->moving.empty()) fail(AIMS_ERR_ARG, "no moving-grid model set (aims_grid_set_moving)");
    for (int k = 0; k < g->n_sys; ++k)
      if (!g->moving[k]) fail(AIMS_ERR_ARG, "system %d has no moving-grid model", k);
    require_device(P, "P", (size_t)g->mat_total * sizeof(double));
    require_device(gE, "gE", sizeof(double));
    require_device(dE_dR, "dE_dR", 3 * (size_t)g->n_atoms * sizeof(double));
    debug_check_symmetric(g, P, "P");
    if (sums_out_or_null) require_device(sums_out_or_null, "sums_out", 3 * (size_t)g->n_sys * sizeof(double));
    set_positions(g, nullptr);
    if (g->moved) fail(AIMS_ERR_ARG, "total forces are taken at the setup positions");
    int max_na = 1;
    for (int k = 0; k < g->n_sys; ++k)
      max_na = std::max(max_na, (int)(g->sys_atom_range[2 * k + 1] - g->sys_atom_range[2 * k]));
    if (3 * (size_t)max_na * sizeof(double) > 64 * 1024)
      fail(AIMS_ERR_UNSUPPORTED, "total forces support up to %d atoms per system", (int)(64 * 1024 / 24));
    if (max_na <= kForceWaveMaxAtoms && !g->gf_ready) build_force_tables(g, max_na);
    hipStream_t st = g->stream;
    BatchSet& bs = g->dens;
    if (g->slab_cap34 < bs.slab_elems) {
      if (g->d_slab3) g->release(g->d_slab3);
      if (g->d_slab4) g->release(g->d_slab4);
      g->d_slab3 = g->d_slab4 = nullptr;
      g->slab_cap34 = 0;
      g->d_slab3 = g->alloc(bs.slab_elems * sizeof(double));
      g->d_slab4 = g->alloc(bs.slab_elems * sizeof(double));
      g->slab_cap34 = bs.slab_elems;
    }
    if (!g->d_ntmp) {
      g->d_ntmp = (double*)g->alloc(std::max<int64_t>(1, g->n_points) * sizeof(double));
      g->d_sums_tmp = (double*)g->alloc(3 * (size_t)g->n_sys * sizeof(double));
    }
    const size_t n = (size_t)g->n_points;
    const bool mixed = prec != AIMS_FP64;
    hipchk(launch_vext(bs.dv, g->n_points, g->d_pt_sys, g->d_sys_natoms, g->d_Z, g->d_sys_model,
                       g->d_vmodel, st), "model potential");
    if (mixed) hipchk(launch_convert_f32(P, g->d_P32, (size_t)g->mat_total, st), "convert P");
    hipchk(launch_fill(g->d_n_sorted, n, 0.0, st), "fill n");
    hipchk(launch_fill(g->d_dsorted, n, 0.0, st), "fill D");
    hipchk(launch_fill(g->d_gpt, 3 * n, 0.0, st), "fill point sums");
    hipchk(launch_fill(g->d_et_batch, bs.batches.size(), 0.0, st), "fill E_T");
    hipchk(launch_fill(dE_dR, 3 * (size_t)g->n_atoms, 0.0, st), "fill dE/dR");
    const double* v = g->d_vmodel;
    const ItemList& L = tile_list(g, bs, dens_key_of(g, prec));
    for (size_t gi = 0; gi < bs.groups.size(); ++gi) {
      const auto& gr = bs.groups[gi];
      const int nbt = gr.b1 - gr.b0;
      if (!mixed) {
        double *s1 = (double*)g->d_slab1, *s2 = (double*)g->d_slab2;
        double *s3 = (double*)g->d_slab3, *s4 = (double*)g->d_slab4;
        timed(g, kProfPhi, 0.0, "phi_eval", [&] {
          return launch_phi_eval<double>(bs.dv, gr.b0, nbt, kModeDensity, nullptr, s1, s2, st);
        });
        for (const auto& run : L.runs[gi]) {
          const int nit = (int)(run.i1 - run.i0);
          timed(g, kProfBackward, gr.flops / L.runs[gi].size(), "X", [&] {
            return launch_density<double>(bs.dv, run.nbn, L.d_items + run.i0, nit, P, s1, s2,
                                          g->d_n_sorted, g->d_et_batch, st, s3, Queue(), g->d_dsorted);
          });
          timed(g, kProfBackward, gr.flops / L.runs[gi].size(), "Y", [&] {
            return launch_density<double>(bs.dv, run.nbn, L.d_items + run.i0, nit, P, s2, s2, nullptr,
                                          nullptr, st, s4);
          });
        }
        timed(g, kProfBackward, 0.0, "pulay", [&] {
          return launch_pulay<double>(bs.dv, gr.b0, nbt, v, s3, s4, gE, dE_dR, st, g->d_gpt);
        });
      } else {
        float *s1 = (float*)g->d_slab1, *s2 = (float*)g->d_slab2;
        float *s3 = (float*)g->d_slab3, *s4 = (float*)g->d_slab4;
        timed(g, kProfPhi, 0.0, "phi_eval", [&] {
          return launch_phi_eval<float>(bs.dv, gr.b0, nbt, kModeDensity, nullptr, s1, s2, st);
        });
        for (const auto& run : L.runs[gi]) {
          const int nit = (int)(run.i1 - run.i0);
          timed(g, kProfBackward, gr.flops / L.runs[gi].size(), "X", [&] {
            return launch_density<float>(bs.dv, run.nbn, L.d_items + run.i0, nit, g->d_P32, s1, s2,
                                         g->d_n_sorted, g->d_et_batch, st, s3, Queue(), g->d_dsorted);
          });
          timed(g, kProfBackward, gr.flops / L.runs[gi].size(), "Y", [&] {
            return launch_density<float>(bs.dv, run.nbn, L.d_items + run.i0, nit, g->d_P32, s2, s2,
                                         nullptr, nullptr, st, s4);
          });
        }
        timed(g, kProfBackward, 0.0, "pulay", [&] {
          return launch_pulay<float>(bs.dv, gr.b0, nbt, v, s3, s4, gE, dE_dR, st, g->d_gpt);
        });
      }
    }
    if (max_na <= kForceWaveMaxAtoms && !g->force_thread_path) {
      timed(g, kProfBackward, 0.0, "grid", [&] {
        return launch_gridforce_wave(bs.dv, g->gf_k, g->d_franges, g->gf_nranges, max_na,
                                     g->d_sys_natoms, g->d_Z, g->d_sys_model, g->d_pair_off,
                                     g->d_inv_aR, g->d_owner, g->d_vmodel, g->d_n_sorted,
                                     g->d_dsorted, g->d_gpt, g->d_fpart, g->d_fpart_off,
                                     g->d_fnrange, gE, dE_dR, st);
      });
    } else {
      timed(g, kProfBackward, 0.0, "grid", [&] {
        return launch_gridforce(bs.dv, (int)bs.batches.size(), max_na, g->d_sys_natoms, g->d_Z,
                                g->d_sys_model, g->d_owner, g->d_wgrid, g->d_vmodel, g->d_n_sorted,
                                g->d_dsorted, g->d_gpt, gE, dE_dR, st);
      });
    }
    if (sums_out_or_null) {
      hipchk(launch_density_finish(bs.dv, g->d_n_sorted, v, g->d_ntmp, g->d_part, g->nblk_finish,
                                   g->d_et_batch, sums_out_or_null, st), "sums");
    }
  });
}

aims_status aims_density_matrix(aims_grid* g, int32_t method, const double* H, const double* S,
                                const double* n_electrons, double kT, double* P_out,
                                double* eps_out_or_null, double* mu_out_or_null) {
  return guarded(__func__, g, [&] {
    if (method != AIMS_DM_EIGEN && method != AIMS_DM_PURIFY) fail(AIMS_ERR_ARG, "unknown method %d", method);
    if (!n_electrons) fail(AIMS_ERR_ARG, "null n_electrons");
    if (!(kT >= 0.0) || !std::isfinite(kT)) fail(AIMS_ERR_ARG, "kT must be finite and >= 0");
    require_device(H, "H", (size_t)g->mat_total * sizeof(double));
    require_device(S, "S", (size_t)g->mat_total * sizeof(double));
    require_device(P_out, "P_out", (size_t)g->mat_total * sizeof(double));
    if (eps_out_or_null) {
      if (method == AIMS_DM_PURIFY) fail(AIMS_ERR_UNSUPPORTED, "purification computes no eigenvalues (eps_out must be NULL)");
      require_device(eps_out_or_null, "eps_out", (size_t)g->nb_total * sizeof(double));
    }
    for (int k = 0; k < g->n_sys; ++k) {
      const double ne = n_electrons[k];
      const int nb = g->systems[k].nb;
      if (!std::isfinite(ne) || ne < 0.0 || ne > 2.0 * nb)
        fail(AIMS_ERR_ARG, "system %d: %g electrons do not fit %d states", k, ne, nb);
      if (method == AIMS_DM_PURIFY) {
        if (kT != 0.0) fail(AIMS_ERR_UNSUPPORTED, "purification takes aufbau occupations (kT = 0)");
        if (ne != 2.0 * std::floor(ne / 2.0))
          fail(AIMS_ERR_UNSUPPORTED, "system %d: purification needs an even electron count (got %g)", k, ne);
      }
    }
    g->dm.stream = g->stream;
    int64_t eoff = 0;
    for (int k = 0; k < g->n_sys; ++k) {
      const int nb = g->systems[k].nb;
      const int64_t off = g->systems[k].mat_off;
      double mu = 0.0;
      std::string err;
      const int rc = dm_solve(g->dm, method, nb, H + off, S + off, n_electrons[k], kT, P_out + off,
                              eps_out_or_null ? eps_out_or_null + eoff : nullptr, &mu, err);
      if (rc) fail((aims_status)rc, "system %d: %s", k, err.c_str());
      if (mu_out_or_null) mu_out_or_null[k] = mu;
      eoff += nb;
    }
    g->dm_iterations = g->dm.last_iterations;
  });
}

aims_status aims_grid_set_hartree(aims_grid* g, int32_t sys, const aims_hartree_grid* h) {
  return guarded(__func__, g, [&] {
    if (!h) fail(AIMS_ERR_ARG, "null Hartree grid description");
    if (sys < 0 || sys >= g->n_sys) fail(AIMS_ERR_ARG, "system %d out of range", sys);
    if (h->n_radial < 3 || h->n_radial > 4096) fail(AIMS_ERR_ARG, "n_radial must be in 3..4096");
    if (!(h->r_map > 0.0) || !std::isfinite(h->r_map)) fail(AIMS_ERR_ARG, "r_map must be > 0");
    if (h->l_max < 0 || h->l_max > kHartreeMaxL)
      fail(AIMS_ERR_UNSUPPORTED, "l_max must be in 0..%d", kHartreeMaxL);
    if (g->hartree_lmax >= 0 && h->l_max != g->hartree_lmax)
      fail(AIMS_ERR_ARG, "every system of a handle takes the same l_max (%d)", g->hartree_lmax);
    const int64_t p0 = g->sys_pt_range[2 * sys], p1 = g->sys_pt_range[2 * sys + 1];
    const int a0 = (int)g->sys_atom_range[2 * sys], a1 = (int)g->sys_atom_range[2 * sys + 1];
    if (p1 > p0 && (!h->pt_owner || !h->pt_node)) fail(AIMS_ERR_ARG, "null point arrays");
    for (int64_t i = 0; i < p1 - p0; ++i) {
      if (h->pt_owner[i] < 0 || h->pt_owner[i] >= a1 - a0)
        fail(AIMS_ERR_ARG, "pt_owner[%lld] = %d out of range", (long long)i, h->pt_owner[i]);
      if (h->pt_node[i] < 0 || h->pt_node[i] >= h->n_radial)
        fail(AIMS_ERR_ARG, "pt_node[%lld] = %d out of range", (long long)i, h->pt_node[i]);
    }
    if (g->h_K.empty()) {
      g->h_K.assign(g->n_sys, 0);
      g->h_rmap.assign(g->n_sys, 0.0);
      g->h_owner.assign(g->n_points, 0);
      g->h_node.assign(g->n_points, 0);
    }
    for (int64_t i = p0; i < p1; ++i) {
      const int64_t q = g->perm_host[i] - p0;     // caller index within the system
      g->h_owner[i] = a0 + h->pt_owner[q];
      g->h_node[i] = h->pt_node[q];
    }
    g->h_K[sys] = h->n_radial;
    g->h_rmap[sys] = h->r_map;
    g->hartree_lmax = h->l_max;
    g->h_ready = false;
  });
}


aims_status aims_hartree(aims_grid* g, const double* n, double* v_out, double* E_out_or_null) {
  return guarded(__func__, g, [&] {
    if (g->h_K.empty()) fail(AIMS_ERR_ARG, "no Hartree grid set (aims_grid_set_hartree)");
    for (int k = 0; k < g->n_sys; ++k)
      if (!g->h_K[k]) fail(AIMS_ERR_ARG, "system %d has no Hartree grid", k);
    require_device(n, "n", (size_t)g->n_points * sizeof(double));
    require_device(v_out, "v_out", (size_t)g->n_points * sizeof(double));
    if (E_out_or_null) require_device(E_out_or_null, "E_out", (size_t)g->n_sys * sizeof(double));
    set_positions(g, nullptr);
    if (g->moved) fail(AIMS_ERR_ARG, "the Hartree potential is taken at the setup positions");
    if (!g->h_ready) build_hartree(g);
    hipchk(launch_hartree(g->dens.dv, g->hd, n, v_out, E_out_or_null, g->stream), "Hartree");
  });
}

aims_status aims_xc_gga(aims_grid* g, int32_t functional, const double* n, const double* grad_n,
                        double* v_out, double* u_out, double* sums_out_or_null) {
  return guarded(__func__, g, [&] {
    if (functional != AIMS_XC_PBE) fail(AIMS_ERR_UNSUPPORTED, "aims_xc_gga takes AIMS_XC_PBE");
    require_device(n, "n", (size_t)g->n_points * sizeof(double));
    require_device(grad_n, "grad_n", 3 * (size_t)g->n_points * sizeof(double));
    require_device(v_out, "v_out", (size_t)g->n_points * sizeof(double));
    require_device(u_out, "u_out", 3 * (size_t)g->n_points * sizeof(double));
    if (sums_out_or_null) require_device(sums_out_or_null, "sums_out", 2 * (size_t)g->n_sys * sizeof(double));
    if (!g->d_xc_part) g->d_xc_part = (double*)g->alloc(2 * (size_t)kXcBlocks * g->n_sys * sizeof(double));
    hipchk(launch_pbe(g->dens.dv, n, grad_n, v_out, u_out, g->d_xc_part, sums_out_or_null, g->stream),
           "xc");
  });
}

aims_status aims_density_gradient(aims_grid* g, const double* P, double* n_out_or_null,
                                  double* grad_out) {
  return guarded(__func__, g, [&] {
    require_device(P, "P", (size_t)g->mat_total * sizeof(double));
    require_device(grad_out, "grad_out", 3 * (size_t)g->n_points * sizeof(double));
    debug_check_symmetric(g, P, "P");
    if (n_out_or_null) require_device(n_out_or_null, "n_out", (size_t)g->n_points * sizeof(double));
    set_positions(g, nullptr);
    if (g->moved) fail(AIMS_ERR_ARG, "the density gradient is taken at the setup positions");
    hipStream_t st = g->stream;
    BatchSet& bs = g->dens;
    if (g->slab_cap34 < bs.slab_elems) {
      if (g->d_slab3) g->release(g->d_slab3);
      if (g->d_slab4) g->release(g->d_slab4);
      g->d_slab3 = g->d_slab4 = nullptr;
      g->slab_cap34 = 0;
      g->d_slab3 = g->alloc(bs.slab_elems * sizeof(double));
      g->d_slab4 = g->alloc(bs.slab_elems * sizeof(double));
      g->slab_cap34 = bs.slab_elems;
    }
    if (!g->d_ntmp) {
      g->d_ntmp = (double*)g->alloc(std::max<int64_t>(1, g->n_points) * sizeof(double));
      g->d_sums_tmp = (double*)g->alloc(3 * (size_t)g->n_sys * sizeof(double));
    }
    hipchk(launch_fill(g->d_n_sorted, (size_t)g->n_points, 0.0, st), "fill n");
    hipchk(launch_fill(g->d_et_batch, bs.batches.size(), 0.0, st), "fill E_T");
    const ItemList& L = tile_list(g, bs, dens_key_of(g, AIMS_FP64));
    double *s1 = (double*)g->d_slab1, *s2 = (double*)g->d_slab2, *s3 = (double*)g->d_slab3;
    for (size_t gi = 0; gi < bs.groups.size(); ++gi) {
      const auto& gr = bs.groups[gi];
      const int nbt = gr.b1 - gr.b0;
      timed(g, kProfPhi, 0.0, "phi_eval", [&] {
        return launch_phi_eval<double>(bs.dv, gr.b0, nbt, kModeDensity, nullptr, s1, s2, st);
      });
      for (const auto& run : L.runs[gi]) {
        const int nit = (int)(run.i1 - run.i0);
        timed(g, kProfDensity, gr.flops / L.runs[gi].size(), "X", [&] {
          return launch_density<double>(bs.dv, run.nbn, L.d_items + run.i0, nit, P, s1, s2,
                                        g->d_n_sorted, g->d_et_batch, st, s3);
        });
      }
      hipchk(launch_gradn(bs.dv, gr.b0, nbt, s3, grad_out, st), "density gradient");
    }
    if (n_out_or_null)
      hipchk(launch_density_finish(bs.dv, g->d_n_sorted, nullptr, n_out_or_null, g->d_part,
                                   g->nblk_finish, g->d_et_batch, g->d_sums_tmp, st),
             "density");
  });
}

aims_status aims_xc(aims_grid* g, int32_t functional, const double* n, double* v_xc_out,
                    double* sums_out_or_null) {
  return guarded(__func__, g, [&] {
    if (functional == AIMS_XC_PBE) fail(AIMS_ERR_UNSUPPORTED, "PBE needs the density gradient (aims_xc_gga)");
    if (functional != AIMS_XC_LDA_PW92) fail(AIMS_ERR_UNSUPPORTED, "unknown functional %d", functional);
    require_device(n, "n", (size_t)g->n_points * sizeof(double));
    require_device(v_xc_out, "v_xc_out", (size_t)g->n_points * sizeof(double));
    if (sums_out_or_null) require_device(sums_out_or_null, "sums_out", 2 * (size_t)g->n_sys * sizeof(double));
    if (!g->d_xc_part) g->d_xc_part = (double*)g->alloc(2 * (size_t)kXcBlocks * g->n_sys * sizeof(double));
    hipchk(launch_lda(g->dens.dv, n, v_xc_out, g->d_xc_part, sums_out_or_null, g->stream), "xc");
  });
}

struct aims_step_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
};

aims_status aims_step_graph_create(aims_grid* g, aims_precision prec, const double* P, const double* v,
                                   double* n_out, double* sums_out, double* H, aims_step_graph** out) {
  return guarded(__func__, g, [&] {
    if (!out) fail(AIMS_ERR_ARG, "out is NULL");
    *out = nullptr;
    check_prec(prec);
    require_device(P, "P", (size_t)g->mat_total * sizeof(double));
    require_device(v, "v", (size_t)g->n_points * sizeof(double));
    require_device(n_out, "n_out", (size_t)g->n_points * sizeof(double));
    require_device(sums_out, "sums_out", 3 * (size_t)g->n_sys * sizeof(double));
    debug_check_symmetric(g, P, "P");
    require_device(H, "H", (size_t)g->mat_total * sizeof(double));
    set_positions(g, nullptr);
    if (!g->stream) fail(AIMS_ERR_ARG, "step graphs need a non-default stream at setup");
    if (g->profiling) fail(AIMS_ERR_ARG, "disable profiling before capturing a step graph");
    if (prec == AIMS_INT8X7)   // buffers taken before the capture begins
      prepare_i8(g, &hset(g, g->h_merge[AIMS_INT8X7], g->h_ratio[AIMS_INT8X7]));
    std::unique_ptr<aims_step_graph> sg(new aims_step_graph());
    sg->stream = g->stream;
    g->graph_captured = true;
    hipchk(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      density_call(g, prec, P, v, n_out, sums_out);
      hs_call(g, prec, kModeH, v, H);
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(g->stream, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    hipchk(hipStreamEndCapture(g->stream, &sg->graph), "end capture");
    hipchk(hipGraphInstantiate(&sg->exec, sg->graph, nullptr, nullptr, 0), "instantiate");
    *out = sg.release();
  });
}

aims_status aims_step_graph_launch(aims_step_graph* graph) {
  if (!graph || !graph->exec) return AIMS_ERR_ARG;
  return hipGraphLaunch(graph->exec, graph->stream) == hipSuccess ? AIMS_OK : AIMS_ERR_HIP;
}

void aims_step_graph_destroy(aims_step_graph* graph) {
  if (!graph) return;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
}

aims_status aims_profile_enable(aims_grid* g, int on) {
  return guarded(__func__, g, [&] {
    prof_collect(g);
    g->profiling = on != 0;
    for (int k = 0; k < 6; ++k) {
      g->prof_count[k] = 0;
      g->prof_ms[k] = 0.0;
      g->prof_work[k] = 0.0;
    }
  });
}

aims_status aims_profile_read(aims_grid* g, const char* kernel, int64_t* launches, double* total_ms,
                              double* work) {
  return guarded(__func__, g, [&] {
    if (!kernel) fail(AIMS_ERR_ARG, "kernel name is NULL");
    int k = -1;
    for (int i = 0; i < 6; ++i)
      if (strcmp(kernel, kProfNames[i]) == 0) k = i;
    if (k < 0) fail(AIMS_ERR_ARG, "unknown kernel family '%s'", kernel);
    prof_collect(g);
    if (launches) *launches = g->prof_count[k];
    if (total_ms) *total_ms = g->prof_ms[k];
    if (work) *work = g->prof_work[k];
  });
}

aims_status aims_get_tuning(const aims_grid* g, aims_precision prec, aims_tuning* out) {
  if (!g || !out || prec < AIMS_FP64 || prec > AIMS_INT8X7) return AIMS_ERR_ARG;
  memset(out, 0, sizeof(*out));
  out->h_merge = g->h_merge[prec];
  out->h_flops_per_atomic = g->h_ratio[prec];
  out->density_pblocks = g->d_pblocks[prec];
  out->persistent = g->persistent[prec];
  out->h_tile32_mask = (int32_t)g->h_tile32[prec];
  for (int b = 0; b < kDensityBuckets; ++b) out->density_bucket_pblocks[b] = g->d_bucket_pblocks[prec][b];
  return AIMS_OK;
}

aims_status aims_set_tuning(aims_grid* g, aims_precision prec, const aims_tuning* t) {
  return guarded(__func__, g, [&] {
    if (!t || prec < AIMS_FP64 || prec > AIMS_INT8X7) fail(AIMS_ERR_ARG, "bad tuning arguments");
    if (t->h_merge < 0 || t->h_merge > 4) fail(AIMS_ERR_ARG, "h_merge must be in 0..4");
    if (t->density_pblocks < 2 || t->density_pblocks > 5) fail(AIMS_ERR_ARG, "density_pblocks must be in 2..5");
    if (t->persistent != 0 && t->persistent != 1) fail(AIMS_ERR_ARG, "persistent must be 0 or 1");
    if (t->h_flops_per_atomic < 0 || t->h_flops_per_atomic > (1 << 20))
      fail(AIMS_ERR_ARG, "h_flops_per_atomic must be in 0..2^20");
    for (int b = 0; b < kDensityBuckets; ++b)
      if (t->density_bucket_pblocks[b] != 0 && (t->density_bucket_pblocks[b] < 2 || t->density_bucket_pblocks[b] > 5))
        fail(AIMS_ERR_ARG, "density_bucket_pblocks[%d] must be 0 or in 2..5", b);
    if (t->h_tile32_mask < 0 || t->h_tile32_mask >= (1 << (2 * kDensityBuckets)))
      fail(AIMS_ERR_ARG, "h_tile32_mask must be in 0..2^%d - 1", 2 * kDensityBuckets);
    if (t->h_tile32_mask && prec != AIMS_FP64 && prec != AIMS_FP32)
      fail(AIMS_ERR_UNSUPPORTED, "32 x 32 H tiles exist for AIMS_FP64 and AIMS_FP32");
    BatchSet& hb = hset(g, t->h_merge, t->h_flops_per_atomic);
    tile_list(g, hb, h_key((uint32_t)t->h_tile32_mask));
    if (prec != AIMS_INT8X7) tile_list(g, g->dens, density_key(t->density_pblocks, t->density_bucket_pblocks));
    g->h_merge[prec] = t->h_merge;
    g->h_ratio[prec] = t->h_flops_per_atomic;
    g->persistent[prec] = t->persistent;
    g->d_pblocks[prec] = t->density_pblocks;
    g->h_tile32[prec] = (uint32_t)t->h_tile32_mask;
    for (int b = 0; b < kDensityBuckets; ++b) g->d_bucket_pblocks[prec][b] = t->density_bucket_pblocks[b];
  });
}

// Per tile-shape bucket: the batches and the algorithmic flops (2 n_p n_b^2) of the density
// partition (which = 0, kDensityBuckets buckets) or of the precision's H partition (which = 1,
// 2 kDensityBuckets buckets).
aims_status aims_bucket_stats(aims_grid* g, aims_precision prec, int32_t which, int64_t* batches_out,
                              double* flops_out) {
  return guarded(__func__, g, [&] {
    check_prec(prec);
    if (which != 0 && which != 1) fail(AIMS_ERR_ARG, "which must be 0 (density) or 1 (H)");
    if (!batches_out || !flops_out) fail(AIMS_ERR_ARG, "null output");
    const int nbk = which ? 2 * kDensityBuckets : kDensityBuckets;
    for (int b = 0; b < nbk; ++b) {
      batches_out[b] = 0;
      flops_out[b] = 0.0;
    }
    const BatchSet& bs = which ? hset(g, g->h_merge[prec], g->h_ratio[prec]) : g->dens;
    for (const BatchDesc& d : bs.batches) {
      const int b = which ? h_bucket(d.n_b) : density_bucket(d.n_b);
      batches_out[b] += 1;
      flops_out[b] += 2.0 * d.n_p * (double)d.n_b * d.n_b;
    }
  });
}

aims_status aims_positions_status(aims_grid* g) {
  return guarded(__func__, g, [&] {
    int flag = 0;
    hipchk(hipMemcpyAsync(&flag, g->d_pos_flag, sizeof(int), hipMemcpyDeviceToHost, g->stream), "status");
    hipchk(hipStreamSynchronize(g->stream), "status");
    if (flag) fail(AIMS_ERR_STALE, "the last positions given on the device moved an atom beyond screen_margin "
                                   "(or were not finite); that call's outputs are NaN");
  });
}

aims_status aims_work_stats(const aims_grid* g, int64_t* n_batches, double* sum_np_nb2, double* sum_nb2) {
  if (!g) return AIMS_ERR_ARG;
  if (n_batches) *n_batches = (int64_t)g->dens.batches.size();
  if (sum_np_nb2) *sum_np_nb2 = g->dens.sum_np_nb2;
  if (sum_nb2) *sum_nb2 = g->dens.sum_nb2;
  return AIMS_OK;
}

int64_t aims_n_basis(const aims_grid* g) { return g ? g->nb_total : -1; }
int64_t aims_n_points(const aims_grid* g) { return g ? g->n_points : -1; }
int32_t aims_n_atoms(const aims_grid* g) { return g ? g->n_atoms : -1; }

const char* aims_last_error(const aims_grid* g) { return g ? g->err.c_str() : g_setup_error.c_str(); }

int32_t aims_last_purify_products(const aims_grid* g) { return g ? g->dm_iterations : 0; }

void aims_grid_destroy(aims_grid* g) { delete g; }

}  // extern "C"
