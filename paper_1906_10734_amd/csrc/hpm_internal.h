// Internal plan layout and launcher declarations of the HPM library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hpm.h"

namespace hpm {

constexpr int kMaxLevelsHost = 11;  // levels 0..10

// The tree build's level table (device memory; also copied to the mailbox words from
// Plan::kBoxLev on): first cell id and cell count of each level (offsets past the last level are
// the cell total), the cell and leaf totals, the leaves of levels 0 and 1, the first leaf-list
// index of each level, and where each level starts in the list of split cells of levels >= 1.
constexpr int kLevOff = 0, kLevCnt = 16, kLevCells = 32, kLevLeaves = 33, kLevLeavesLt2 = 34,
              kLevLeafOff = 40, kLevSplitOff = 52, kLevWords = 64;

struct HpmError {
  hpm_status status;
  std::string msg;
};

void set_last_error(const std::string& msg);
[[noreturn]] void fail(hpm_status s, const std::string& msg);

// Runs f and turns a thrown HpmError (or a host allocation failure) into its status; the message
// goes to the calling thread's last error.
template <typename F>
hpm_status guarded(F&& f) {
  try {
    f();
    return HPM_OK;
  } catch (const HpmError& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return HPM_ERR_NO_MEMORY;
  } catch (...) {
    set_last_error("unexpected exception");
    return HPM_ERR_DEVICE;
  }
}

#define HPM_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      ::hpm::fail(e_ == hipErrorOutOfMemory ? HPM_ERR_NO_MEMORY : HPM_ERR_DEVICE,           \
                  std::string(#call) + ": " + hipGetErrorString(e_));                       \
  } while (0)

#define HPM_LAUNCH_CHECK() HPM_HIP(hipGetLastError())

// A fixed region of device memory that buffers are carved from instead of hipMalloc, for the
// entry point that allocates nothing (bump allocation, 256-byte aligned, nothing is returned until
// the region is dropped as a whole).
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
  void* take(size_t b);
};

// The arena that DevBuf allocations of the calling thread come from (null: hipMalloc). Set for
// the duration of a no-allocation call by ArenaScope.
extern thread_local Arena* t_arena;
struct ArenaScope {
  Arena* prev;
  explicit ArenaScope(Arena* a) : prev(t_arena) { t_arena = a; }
  ~ArenaScope() { t_arena = prev; }
};

// A device allocation that frees itself (from hipMalloc, or from the thread's arena when one is
// set, in which case release() only forgets it).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool in_arena = false;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p && !in_arena) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    in_arena = false;
  }
  static void* take(size_t b, bool* from_arena) {
    void* q = nullptr;
    *from_arena = t_arena != nullptr;
    if (t_arena) q = t_arena->take(b);
    else HPM_HIP(hipMalloc(&q, b));
    return q;
  }
  // (re)allocate to at least b bytes; contents are not preserved
  void reserve(size_t b) {
    if (b <= bytes && p) return;
    release();
    if (b == 0) b = 16;
    p = take(b, &in_arena);
    bytes = b;
  }
  // grow to at least b bytes, preserving the first "keep" bytes
  void grow(size_t b, size_t keep, hipStream_t s) {
    if (b <= bytes && p) return;
    bool qa = false;
    void* q = take(b, &qa);
    if (p && keep) HPM_HIP(hipMemcpyAsync(q, p, keep, hipMemcpyDeviceToDevice, s));
    HPM_HIP(hipStreamSynchronize(s));
    release();
    p = q;
    bytes = b;
    in_arena = qa;
  }
  template <typename U>
  U* as() const { return static_cast<U*>(p); }
  void swap(DevBuf& o) {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
    std::swap(in_arena, o.in_arena);
  }
};

// The interaction kernel of a problem (hpm_kernel and its screening length).
struct PairKernel {
  int32_t kind = HPM_KERNEL_NEWTON;
  double screening = 0.0;
};

// Constant tables of one (precision, N_g, softening, box, levels) combination, in device memory.
struct Tables {
  DevBuf m2m;    // [2][NG][NG]: T1^a[p][q] = l_p((a + xi_q)/2), a = -1/2 (index 0), +1/2 (1)
  DevBuf l2l;    // [2][NL][NL]: the same on the target gridlet's nodes (equal to m2m unless
                 // the gridlets are extended)
  DevBuf fitw;   // [Kpad][Mpad]: W[n][p] = B^phi[p][n], Legendre-moment fit matrix, zero padded
  DevBuf ghat;   // [levels 2..L][(n/2+1)^3]: octant of the lattice Green transform / n^3
  DevBuf gxy;    // [levels 2..L][4 N_g + 1][n/2+1][n/2+1]: Green function transformed along x
                 // and y only, at z offsets d <= 4 N_g, [d][ky][kx], / n^2
  DevBuf gcell;  // cell-by-cell and shared-transform routes only: [levels 2..L][343 offsets][(2N_g)^2 (N_g+1)] complex,
                 // transform of the cyclic Green array of each source cube offset, / (2 N_g)^3
  DevBuf twff;   // FP32 plans: [8 N_g] e^{+2 pi i m / n} as {cos hi, sin hi, cos lo, sin lo}
  int kpad = 0, mpad = 0;
  int ghat_levels = 0;
  int gcell_levels = 0;
};

struct Plan {
  hpm_problem prob{};
  int prec = HPM_F32;
  int ng = 4;
  int M = 64;       // source gridlet size N_g^3
  int ext = 0;      // 1: extended target gridlets (N_g + 2 nodes per axis)
  int NL = 4;       // target gridlet nodes per axis, N_g + 2 ext
  int ML = 64;      // target gridlet size NL^3 (local potentials)
  int route = HPM_M2L_GRID;  // source-to-target route of the evaluations (an hpm_m2l_mode)
  int64_t n = 0;
  bool valid = false;  // a tree is built and consistent with the buffers
  int depth = 0;  // Morton key depth D
  int nlevels = 0;
  int level_off[kMaxLevelsHost + 1] = {0};
  int64_t ncells = 0;
  int64_t cap_cells = 0;
  int64_t nleaves = 0;
  int64_t nleaves_lt2 = 0;  // leaves at levels 0 and 1 come first in the leaf list
  size_t elem = 4;          // sizeof(real)

  // particles, sorted by key
  DevBuf keys, perm, xs, ys, zs, ms;
  // cells (global id space, levels contiguous)
  DevBuf ckey, ccoord, cpb, cpe, cparent, cflags, child8, nbr27;
  DevBuf leaves;
  // virtual cubes (interaction-zone cubes inside coarser leaves), cell ids ncells .. ncells+nvirt-1
  int64_t nvirt = 0;
  DevBuf vcubes;  // [nvirt][3]: cube id (1 << 3l | level-l Morton key), first and end sorted
                  // particle; in the order found
  DevBuf vlevel;  // [nvirt] level
  DevBuf vlist;   // [nvirt] cell id ncells + v
  // the set of virtual cube ids while they are listed: open addressing, 2^vhash_bits slots of
  // (generation << 32 | id, v), grown when a build overflows it; vcount: cubes listed, the set
  // is full
  DevBuf vhash_keys, vhash_vals, vcount;
  int vhash_bits = 0;
  // source gridlet ids of the 216 block slots of each parent of targets (cells of levels
  // 1 .. L-2, from id blocks_first on)
  DevBuf blocks;
  int blocks_first = 0;
  DevBuf dlev;    // the tree build's level table (kLevOff + l: first cell id of level l, the cell
                  // total past the last level)
  // gridlets
  DevBuf gridlet, local, moments;  // gridlet [cells + virtual][M], local [cells][ML]
  // rows of the P2M fit: leaves of levels >= 2, then the virtual cubes (cell ids, levels)
  DevBuf p2m_list, p2m_level;
  int64_t p2m_rows = 0;
  DevBuf lofs;  // [cells][2]: constant part of the local potential (compensated pair)
  DevBuf m2l_mean;          // [cells] double: mean of the source-to-target result, when split
  bool m2l_split = false;   // the source-to-target kernel writes (mean, zero-mean gridlet)
  // FP32 plans on the padded-grid route at N_g = 4 and 6: the source-to-target kernel's inverse
  // x sums and mean, and L2L's constant, in float-float arithmetic instead of double (the mean
  // is then stored as a float pair in m2l_mean's slot)
  bool fp32_strict = false;
  bool m2l_mean_ff = false;  // m2l_mean holds float pairs (set by the kernel launch)
  // near-zone lists and the P2P work items (see downsweep.hip)
  DevBuf near_rb, near_re, item_cnt, item_off, items, partial, pairs;
  DevBuf leaf_of;  // [n] leaf list index of each sorted particle
  DevBuf near_group_items;  // per workgroup of the near-list kernel: item total, then its base
  int near_per_group = 8, near_groups = 1;  // leaves per workgroup of that kernel, workgroups
  int64_t n_items = 0;
  int64_t p2p_pairs = 0;
  int m2l_slots = 0;  // workgroups of a source-to-target launch
  // cell-by-cell route: source spectra [cells of levels >= 2, then virtual cubes][modes] and the
  // accumulated target spectra [cells of levels >= 2][modes]
  DevBuf cell_src, cell_tgt;
  // the split parents (cells of levels 1 .. L-2 with children) in id order, and where each
  // parent level starts in that list (cell_pbeg[L-1] is its length)
  DevBuf cell_plist;
  int cell_pbeg[kMaxLevelsHost + 1] = {0};
  Tables tab;
  // scratch for the tree build: sort buffers and state, per-workgroup level counts, and the hash of cube
  // id -> cell id (slots tagged with the build's generation, so that a new build needs no
  // clearing)
  DevBuf tmp_keys, tmp_vals, sort_ctr, sort_status, tree_blk, chash_slot, chash_val;
  bool sort_clean = false;  // the sort state is all zero (false: clear it before the next sort)
  int chash_bits = 0;
  uint32_t tree_gen = 0;
  // pinned, device-mapped words that kernels write and the host reads after a stream
  // synchronisation (counts that size the next step of the build, input error flags)
  static constexpr int kBoxWords = 128;
  static constexpr int kBoxOutOfBox = 0, kBoxNonfinite = 1, kBoxTotal = 2, kBoxLeavesLt2 = 3;
  static constexpr int kBoxCellLevels = 4;  // words 5 .. 4 + L-1: split-parent list bounds
  static constexpr int kBoxLeaves = 16;     // leaf count (read after the first virtual-cube step)
  static constexpr int kBoxVirt = 17;       // virtual cubes listed
  static constexpr int kBoxVirtFull = 18;   // the virtual-cube set overflowed
  static constexpr int kBoxLev = 24;        // words 24 .. 87: copy of the tree's level table
  int* hbox = nullptr;
  int* dbox = nullptr;
  // a plan of the entry point that allocates nothing: its buffers come from an arena, the mailbox
  // words live in device memory (copied to hbox_store by sync_box), and it has no side stream
  // and no timing events
  bool noalloc = false;
  // device bytes the plan may hold once its tree is known (0: no limit): a rebuild whose tree
  // needs more fails with HPM_ERR_NO_MEMORY before the evaluation buffers are sized (the serving
  // runtime sets it from the budget left at admission)
  size_t byte_cap = 0;
  int hbox_store[kBoxWords] = {0};
  // a second stream (default priority) on which the near-zone sums run beside the far-field
  // chain of an execution, with the events that fork it from and join it to the caller's stream
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  bool overlap = true;  // run the near zone on "side" (from kForkMinParticles particles on)

  // stage timing with HIP events (off unless enabled): a ring of pending executions
  static constexpr int kStages = 5;   // P2M, M2M, M2L, L2L, leaves
  static constexpr int kRing = 64;
  bool timing = false;
  bool events_created = false;
  hipEvent_t ev[kRing][kStages + 1] = {};
  hipEvent_t p2p_ev[kRing][2] = {};  // around the near-zone sums, on the stream that runs them
  hipEvent_t tree_ev[2] = {};
  bool tree_pending = false;  // tree_ev holds a timed build not yet added to stage_ms[0]
  int ring_head = 0, ring_count = 0;
  double stage_ms[kStages + 2] = {0};  // [0] tree build, [1..5] execute stages, [6] near zone
  int64_t n_exec = 0, n_build = 0;
  ~Plan();

  // device memory the plan holds (every buffer above and its tables)
  size_t device_bytes() const;
};

// ---- api.cpp ------------------------------------------------------------------------------------
// host checks of a problem description and of a particle count for it (throw HpmError)
constexpr int64_t kNg8MaxParticles = int64_t(1) << 16;
void check_problem(const hpm_problem* pr);
void check_size(const hpm_problem* pr, int64_t n);
// tables, streams and the first tree of a plan; the tree for new positions; one evaluation.
// Plans are independent of each other: distinct plans may be used from distinct host threads.
void create_plan(Plan& p, const hpm_problem* pr, int64_t n, const void* x, const void* y,
                 const void* z, hipStream_t s);
void rebuild_plan(Plan& p, int64_t n, const void* x, const void* y, const void* z, hipStream_t s);
void execute_plan(Plan& p, const void* m, void* phi, void* ax, void* ay, void* az, hipStream_t s);
// an estimate of the device memory of a plan for n particles, made before its tree is known
// (10 n / leaf capacity + 64 cells, or every cell of a uniform tree; one virtual cube per cell;
// the near-zone work of four source chunks per cell)
size_t plan_bytes_estimate(const hpm_problem& pr, int64_t n);

// waits for "s", after copying the mailbox words to the host when they live in device memory
void sync_box(Plan& p, hipStream_t s);
// zeroes mailbox words [w, w + count) before kernels set them
void clear_box(Plan& p, int w, int count, hipStream_t s);

// ---- tables.cpp -------------------------------------------------------------------------------
// tables for levels 2..max_levels-1 (the Green transforms depend on the level, not on the tree)
void build_tables(Plan& p, int max_levels, hipStream_t s);

// ---- tree.hip -----------------------------------------------------------------------------------
// The tree of the current positions: sorted particles, cells, leaf list, neighbourhoods, the set
// of virtual cubes and the near-zone lists, with one host synchronisation (the counts that size
// the rest: levels, cells, leaves, virtual cubes, near-zone work items). Then finish_virtual
// appends the virtual cubes to the cell arrays and builds the per-parent table of block sources.
void build_tree(Plan& p, const void* x, const void* y, const void* z, hipStream_t s);
void finish_virtual(Plan& p, hipStream_t s);

// ---- upsweep.hip --------------------------------------------------------------------------------
void launch_gather_masses(Plan& p, const void* m, hipStream_t s);
void build_p2m_rows(Plan& p, hipStream_t s);
void launch_p2m(Plan& p, hipStream_t s);
void launch_m2m(Plan& p, int level, hipStream_t s);

// ---- m2l.hip -------------------------------------------------------------------------------------
void launch_m2l(Plan& p, hipStream_t s);
// the transform shared by the children of each split parent (outer cubes of its block); writes
// each child's (mean, zero-mean gridlet)
void launch_m2l_parents(Plan& p, hipStream_t s);
// workgroups of a source-to-target launch (*bytes_per_slot: device workspace per workgroup, 0)
int m2l_workspace_slots(int prec, int ng, size_t* bytes_per_slot);

// ---- m2l_cells.hip -------------------------------------------------------------------------------
// modes of one cell spectrum as stored: C^2 (C/2 + 1) with C = 2 N_g + 2 ext, rounded up to a
// multiple of 16
size_t cell_modes(int ng, int ext);
// the list of split parents that the cell-by-cell route visits is written by the tree build;
// read_cell_parents takes its per-level bounds from the mailbox
void read_cell_parents(Plan& p);
void launch_m2l_cells(Plan& p, hipStream_t s);
// the shared-transform route: the central cubes cell by cell, the outer cubes by
// launch_m2l_parents, both added into each target's (mean, zero-mean gridlet)
void launch_m2l_shared(Plan& p, hipStream_t s);

// ---- downsweep.hip -------------------------------------------------------------------------------
// near-zone ranges, work-item counts and offsets of every leaf (enqueued by the tree build before
// its synchronisation: the leaf count is read on the device), then the work items themselves
void enqueue_near_lists(Plan& p, hipStream_t s);
void finish_near_lists(Plan& p, hipStream_t s);
void launch_l2l(Plan& p, int level, hipStream_t s);
// near-zone partial sums (independent of the far-field chain), then the per-leaf combination
void launch_p2p(Plan& p, hipStream_t s);
void launch_leaf(Plan& p, void* phi, void* ax, void* ay, void* az, hipStream_t s);
void launch_direct_sum(int prec, int64_t n, const void* x, const void* y, const void* z,
                       const void* m, int64_t nt, const int32_t* targets, double G, double eps,
                       PairKernel ker, double* phi, double* ax, double* ay, double* az,
                       hipStream_t s);

}  // namespace hpm

struct hpm_plan_s {
  hpm::Plan p;
};
