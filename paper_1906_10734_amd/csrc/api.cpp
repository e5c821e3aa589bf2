// C ABI of the HPM library: argument checks, plan lifetime, the order of the method's steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "hpm_internal.h"

namespace hpm {

static thread_local std::string g_last_error;
thread_local Arena* t_arena = nullptr;

void* Arena::take(size_t b) {
  const size_t off = (used + 255) & ~size_t(255);
  if (off > size || b > size - off)
    fail(HPM_ERR_NO_MEMORY, "the no-allocation scratch region is exhausted (" +
                                std::to_string(size >> 20) + " MiB)");
  used = off + b;
  return base + off;
}

void sync_box(Plan& p, hipStream_t s) {
  if (p.noalloc)
    HPM_HIP(hipMemcpyAsync(p.hbox, p.dbox, Plan::kBoxWords * sizeof(int), hipMemcpyDeviceToHost, s));
  HPM_HIP(hipStreamSynchronize(s));
}

void clear_box(Plan& p, int w, int count, hipStream_t s) {
  for (int k = 0; k < count; ++k) p.hbox[w + k] = 0;
  if (p.noalloc) HPM_HIP(hipMemsetAsync(p.dbox + w, 0, size_t(count) * sizeof(int), s));
}

void set_last_error(const std::string& msg) { g_last_error = msg; }
void fail(hpm_status s, const std::string& msg) { throw HpmError{s, msg}; }

static void check_kernel(int32_t kernel, double screening) {
  if (kernel != HPM_KERNEL_NEWTON && kernel != HPM_KERNEL_YUKAWA)
    fail(HPM_ERR_INVALID_ARG, "kernel must be HPM_KERNEL_NEWTON or HPM_KERNEL_YUKAWA");
  if (kernel == HPM_KERNEL_YUKAWA && !(std::isfinite(screening) && screening > 0.0))
    fail(HPM_ERR_INVALID_ARG, "the Yukawa kernel needs screening > 0");
}

void check_problem(const hpm_problem* pr) {
  if (!pr) fail(HPM_ERR_INVALID_ARG, "problem is NULL");
  if (pr->abi != HPM_ABI_VERSION) fail(HPM_ERR_INVALID_ARG, "problem.abi != HPM_ABI_VERSION");
  if (pr->precision != HPM_F32 && pr->precision != HPM_F64)
    fail(HPM_ERR_INVALID_ARG, "precision must be HPM_F32 or HPM_F64");
  const int ng = pr->ng;
  if (ng < 1 || ng > 16) fail(HPM_ERR_INVALID_ARG, "ng out of range");
  if (!(ng == 2 || ng == 3 || ng == 4 || ng == 6 || ng == 8))
    fail(HPM_ERR_UNSUPPORTED, "ng must be one of 2, 3, 4, 6, 8");
  if (!(std::isfinite(pr->box_size) && pr->box_size > 0.0)) fail(HPM_ERR_INVALID_ARG, "box_size must be > 0");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(pr->box_lo[k])) fail(HPM_ERR_INVALID_ARG, "box_lo must be finite");
  if (!(std::isfinite(pr->softening) && pr->softening >= 0.0)) fail(HPM_ERR_INVALID_ARG, "softening must be >= 0");
  if (!(std::isfinite(pr->gconst) && pr->gconst > 0.0)) fail(HPM_ERR_INVALID_ARG, "gconst must be > 0");
  check_kernel(pr->kernel, pr->screening);
  if (pr->m2l_mode != HPM_M2L_GRID && pr->m2l_mode != HPM_M2L_CELLS &&
      pr->m2l_mode != HPM_M2L_SHARED)
    fail(HPM_ERR_INVALID_ARG, "m2l_mode must be HPM_M2L_GRID, HPM_M2L_CELLS or HPM_M2L_SHARED");
  if (pr->extended != 0 && pr->extended != 1) fail(HPM_ERR_INVALID_ARG, "extended must be 0 or 1");
  if (pr->reserved != 0) fail(HPM_ERR_INVALID_ARG, "problem.reserved must be 0");
  if (pr->extended && pr->m2l_mode == HPM_M2L_SHARED)
    fail(HPM_ERR_UNSUPPORTED, "the shared-transform route has no extended gridlets");
  if (pr->extended && pr->m2l_mode == HPM_M2L_GRID && ng != 4 && ng != 6)
    fail(HPM_ERR_UNSUPPORTED, "extended gridlets on the padded-grid route need ng = 4 or 6");
  if (pr->extended && ng == 8)
    fail(HPM_ERR_UNSUPPORTED, "no extended gridlets at ng = 8");
  if (ng == 8 && pr->m2l_mode != HPM_M2L_GRID)
    fail(HPM_ERR_UNSUPPORTED, "ng = 8 is built on the padded-grid route only");
  if (pr->uniform_depth < 0 || pr->uniform_depth > 10) fail(HPM_ERR_INVALID_ARG, "uniform_depth must be 0..10");
  if (pr->uniform_depth == 0) {
    if (pr->leaf_capacity < 1) fail(HPM_ERR_INVALID_ARG, "leaf_capacity must be >= 1");
    if (pr->max_depth < 1 || pr->max_depth > 10) fail(HPM_ERR_INVALID_ARG, "max_depth must be 1..10");
  }
}

void check_size(const hpm_problem* pr, int64_t n) {
  if (n < 1 || n > (int64_t(1) << 30)) fail(HPM_ERR_INVALID_ARG, "n must be in [1, 2^30]");
  // N_g = 8 runs on sets of at most kNg8MaxParticles. A 2^18-particle FP32 solve at N_g = 8 ended
  // in a device memory fault in an earlier version of the library (whose source-to-target kernel
  // kept its line buffer in device memory); a CPU emulation of that version and of this one on
  // the same input found every access in bounds, so no cause is shown and the larger sizes stay
  // off.
  if (pr->ng == 8 && n > kNg8MaxParticles)
    fail(HPM_ERR_UNSUPPORTED, "ng = 8 is limited to 65536 particles (a larger solve faulted in an "
                              "earlier version; cause not shown)");
}

// Adds the elapsed time of a timed tree build still pending to the totals.
static void drain_tree(Plan& p) {
  if (!p.tree_pending) return;
  HPM_HIP(hipEventSynchronize(p.tree_ev[1]));
  float ms = 0.f;
  HPM_HIP(hipEventElapsedTime(&ms, p.tree_ev[0], p.tree_ev[1]));
  p.stage_ms[0] += ms;
  p.n_build += 1;
  p.tree_pending = false;
}

// Device bytes the plan will hold once its evaluation buffers are sized for the tree just built.
static size_t projected_bytes(const Plan& p) {
  auto need = [](const DevBuf& b, size_t bytes) { return bytes > b.bytes ? bytes - b.bytes : size_t(0); };
  const size_t cells = size_t(p.ncells), nv = size_t(p.nvirt), e = p.elem;
  const size_t rows = size_t(std::max<int64_t>(p.nleaves - p.nleaves_lt2 + p.nvirt, 1));
  const size_t items = size_t(std::max<int64_t>(p.n_items, 1));
  const size_t parents = p.nlevels > 2 ? size_t(p.level_off[p.nlevels - 1] - p.level_off[1]) : 0;
  size_t extra = need(p.gridlet, (cells + nv) * p.M * e) + need(p.local, cells * p.ML * e) +
                 need(p.moments, rows * p.tab.kpad * e) + need(p.lofs, cells * 2 * e) +
                 need(p.m2l_mean, cells * 8) + need(p.items, items * 16) +
                 need(p.partial, items * 64 * 5 * e) + need(p.p2m_list, rows * 4) +
                 need(p.p2m_level, rows * 4) + need(p.blocks, parents * 216 * 4) +
                 need(p.vlevel, nv * 4) + need(p.vlist, nv * 4);
  if (int64_t(cells + nv) > p.cap_cells)  // the cell arrays grow for the virtual cubes
    extra += size_t(int64_t(cells + nv) - p.cap_cells) * (6 + 8 + 27) * 4;
  if (p.prob.m2l_mode != HPM_M2L_GRID && p.nlevels > 2) {
    const size_t spec = cell_modes(p.ng, p.ext) * 2 * e;
    const size_t ntg = cells - size_t(p.level_off[2]);
    extra += need(p.cell_src, (ntg + nv + 1) * spec) + need(p.cell_tgt, ntg * spec);
  }
  return p.device_bytes() + extra;
}

void rebuild_plan(Plan& p, int64_t n, const void* x, const void* y, const void* z, hipStream_t s) {
  p.valid = false;
  drain_tree(p);
  if (p.timing) HPM_HIP(hipEventRecord(p.tree_ev[0], s));
  p.n = n;
  build_tree(p, x, y, z, s);
  if (p.byte_cap) {
    const size_t want = projected_bytes(p);
    if (want > p.byte_cap)
      fail(HPM_ERR_NO_MEMORY, "the tree of this set needs " + std::to_string(want) +
                                  " bytes of device memory, more than the " +
                                  std::to_string(p.byte_cap) + " the budget leaves");
  }
  finish_virtual(p, s);
  const size_t cells = size_t(p.ncells);
  p.gridlet.reserve((cells + size_t(p.nvirt)) * p.M * p.elem);
  p.local.reserve(cells * p.ML * p.elem);
  build_p2m_rows(p, s);
  p.moments.reserve(size_t(std::max<int64_t>(p.p2m_rows, 1)) * p.tab.kpad * p.elem);
  p.lofs.reserve(cells * 2 * p.elem);
  p.m2l_mean.reserve(cells * sizeof(double));
  if (p.prob.m2l_mode != HPM_M2L_GRID && p.nlevels > 2) {
    const size_t spec = cell_modes(p.ng, p.ext) * 2 * p.elem;
    const size_t ntg = cells - size_t(p.level_off[2]);
    p.cell_src.reserve((ntg + size_t(p.nvirt) + 1) * spec);  // + a zero row
    p.cell_tgt.reserve(ntg * spec);
    read_cell_parents(p);
  }
  finish_near_lists(p, s);
  if (p.timing) {  // read when the next build starts or the times are asked for
    HPM_HIP(hipEventRecord(p.tree_ev[1], s));
    p.tree_pending = true;
  }
  p.valid = true;
}

void create_plan(Plan& p, const hpm_problem* pr, int64_t n, const void* x, const void* y,
                 const void* z, hipStream_t s) {
  p.prob = *pr;
  p.prec = pr->precision;
  p.ng = pr->ng;
  p.M = pr->ng * pr->ng * pr->ng;
  p.ext = pr->extended;
  p.NL = pr->ng + 2 * p.ext;
  p.ML = p.NL * p.NL * p.NL;
  p.elem = (p.prec == HPM_F32) ? 4 : 8;
  p.route = pr->m2l_mode;
  if (p.noalloc) {
    p.hbox = p.hbox_store;
    p.dbox = static_cast<int*>(t_arena->take(Plan::kBoxWords * sizeof(int)));
  } else {
    HPM_HIP(hipHostMalloc(reinterpret_cast<void**>(&p.hbox), Plan::kBoxWords * sizeof(int),
                          hipHostMallocMapped | hipHostMallocCoherent));
    HPM_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&p.dbox), p.hbox, 0));
    HPM_HIP(hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking));
    HPM_HIP(hipEventCreateWithFlags(&p.fork_ev, hipEventDisableTiming));
    HPM_HIP(hipEventCreateWithFlags(&p.join_ev, hipEventDisableTiming));
  }
  const int depth = pr->uniform_depth > 0 ? pr->uniform_depth : pr->max_depth;
  build_tables(p, depth + 1, s);
  size_t slot_bytes = 0;
  p.m2l_slots = m2l_workspace_slots(p.prec, p.ng, &slot_bytes);
  rebuild_plan(p, n, x, y, z, s);
}

// Adds the elapsed times of the oldest pending execution to the totals.
static void drain_one(Plan& p) {
  const int slot = (p.ring_head - p.ring_count + Plan::kRing) % Plan::kRing;
  HPM_HIP(hipEventSynchronize(p.ev[slot][Plan::kStages]));
  for (int k = 0; k < Plan::kStages; ++k) {
    float ms = 0.f;
    HPM_HIP(hipEventElapsedTime(&ms, p.ev[slot][k], p.ev[slot][k + 1]));
    p.stage_ms[k + 1] += ms;
  }
  float pm = 0.f;
  HPM_HIP(hipEventSynchronize(p.p2p_ev[slot][1]));
  HPM_HIP(hipEventElapsedTime(&pm, p.p2p_ev[slot][0], p.p2p_ev[slot][1]));
  p.stage_ms[Plan::kStages + 1] += pm;
  p.n_exec += 1;
  p.ring_count -= 1;
}

// particles from which the near zone of an execution runs beside the source-to-target step
constexpr int64_t kForkMinParticles = int64_t(1) << 16;

void execute_plan(Plan& p, const void* m, void* phi, void* ax, void* ay, void* az,
                  hipStream_t s) {
  hipEvent_t* ev = nullptr;
  hipEvent_t* pev = nullptr;
  if (p.timing) {
    if (p.ring_count == Plan::kRing) drain_one(p);
    ev = p.ev[p.ring_head];
    pev = p.p2p_ev[p.ring_head];
    p.ring_head = (p.ring_head + 1) % Plan::kRing;
    p.ring_count += 1;
    HPM_HIP(hipEventRecord(ev[0], s));
  }
  launch_gather_masses(p, m, s);
  launch_p2m(p, s);
  if (ev) HPM_HIP(hipEventRecord(ev[1], s));
  for (int l = p.nlevels - 2; l >= 2; --l) launch_m2m(p, l, s);
  if (ev) HPM_HIP(hipEventRecord(ev[2], s));
  // the near zone needs only the tree and the sorted masses: for large problems it runs on the
  // side stream beside the source-to-target step (which leaves ALU and memory slots idle) and
  // the leaf pass waits for it; small ones keep it in line, where the fork costs more than it hides
  const bool fork = p.overlap && p.n >= kForkMinParticles && p.side;
  if (fork) {
    HPM_HIP(hipEventRecord(p.fork_ev, s));
    HPM_HIP(hipStreamWaitEvent(p.side, p.fork_ev, 0));
    if (pev) HPM_HIP(hipEventRecord(pev[0], p.side));
    launch_p2p(p, p.side);
    if (pev) HPM_HIP(hipEventRecord(pev[1], p.side));
    HPM_HIP(hipEventRecord(p.join_ev, p.side));
  }
  if (p.route == HPM_M2L_CELLS) launch_m2l_cells(p, s);
  else if (p.route == HPM_M2L_SHARED) launch_m2l_shared(p, s);
  else launch_m2l(p, s);
  if (ev) HPM_HIP(hipEventRecord(ev[3], s));
  for (int l = 2; l < p.nlevels; ++l) launch_l2l(p, l, s);  // level 2: re-centring only
  if (ev) HPM_HIP(hipEventRecord(ev[4], s));
  if (fork) {
    HPM_HIP(hipStreamWaitEvent(s, p.join_ev, 0));
  } else {
    if (pev) HPM_HIP(hipEventRecord(pev[0], s));
    launch_p2p(p, s);
    if (pev) HPM_HIP(hipEventRecord(pev[1], s));
  }
  launch_leaf(p, phi, ax, ay, az, s);
  if (ev) HPM_HIP(hipEventRecord(ev[5], s));
}

size_t Plan::device_bytes() const {
  const DevBuf* bufs[] = {
      &keys, &perm, &xs, &ys, &zs, &ms, &ckey, &ccoord, &cpb, &cpe, &cparent, &cflags, &child8,
      &nbr27, &leaves, &vcubes, &vlevel, &vlist, &vhash_keys, &vhash_vals, &vcount, &blocks, &dlev, &gridlet,
      &local, &moments, &p2m_list, &p2m_level, &lofs, &m2l_mean, &near_rb, &near_re, &item_cnt,
      &item_off, &items, &partial, &pairs, &leaf_of, &near_group_items, &cell_src, &cell_tgt, &cell_plist,
      &tab.m2m, &tab.l2l, &tab.fitw, &tab.ghat, &tab.gxy, &tab.gcell, &tab.twff,
      &tmp_keys, &tmp_vals, &sort_ctr, &sort_status, &tree_blk, &chash_slot, &chash_val};
  size_t total = 0;
  for (const DevBuf* b : bufs) total += b->bytes;
  return total;
}

size_t plan_bytes_estimate(const hpm_problem& pr, int64_t n) {
  const size_t s = pr.precision == HPM_F32 ? 4 : 8;
  const size_t ng = size_t(pr.ng), nl = ng + 2 * size_t(pr.extended != 0);
  const size_t M = ng * ng * ng, ML = nl * nl * nl, kpad = (M + 3) / 4 * 4;
  const int depth = pr.uniform_depth > 0 ? pr.uniform_depth : pr.max_depth;
  int64_t cells = 0;
  if (pr.uniform_depth > 0) {
    int64_t lvl = 1;
    for (int l = 0; l <= pr.uniform_depth; ++l, lvl *= 8) cells += std::min<int64_t>(lvl, n);
  } else {
    // a tree whose leaves hold just over an eighth of the capacity has about 9.2 n / capacity
    // cells, the most a uniform particle density gives
    cells = std::max<int64_t>(1024, 10 * n / std::max(1, pr.leaf_capacity) + 64);
  }
  const size_t c = size_t(cells), np = size_t(n);
  size_t b = np * (5 * 4 + 4 * s);          // keys, perm, sort scratch, leaf map; sorted x, y, z, m
  b += c * (6 * 4 + 8 * 4 + 27 * 4);        // cell arrays (key, coords, range, parent, flags,
                                            // children, neighbours)
  b += c * (9 * 4 + 3 * 4 + 216 * 4 / 8);   // level scratch, leaf list, block tables of parents
  b += np * 8 + np / 8;                     // radix-sort status words, level counts per workgroup
  b += c * (2 * 12 + 4 * 24);               // cube hash, virtual-cube set
  b += c * (2 * M * s + ML * s + 2 * kpad * s + 2 * s + 8);  // gridlets of cells and virtual
                                                              // cubes, locals, fit rows
  b += c * (27 * 8 + 8 + 4 * (16 + 64 * 5 * s));  // near-zone ranges and work items
  const size_t H = 4 * ng + 1, levels = size_t(std::max(depth - 1, 1));
  b += levels * (H * H * H + (4 * ng + 1) * H * H) * s;  // Green transforms
  if (pr.m2l_mode != HPM_M2L_GRID) {
    const size_t spec = cell_modes(int(ng), pr.extended) * 2 * s;
    b += (2 * c + 1) * spec + levels * 343 * spec + 3 * 4 * c;
  }
  return b + (size_t(1) << 20);
}

Plan::~Plan() {
  if (side) {
    (void)hipStreamSynchronize(side);
    (void)hipStreamDestroy(side);
  }
  if (fork_ev) (void)hipEventDestroy(fork_ev);
  if (join_ev) (void)hipEventDestroy(join_ev);
  if (hbox && !noalloc) (void)hipHostFree(hbox);
  if (events_created) {
    for (auto& set : ev)
      for (auto& e : set)
        if (e) (void)hipEventDestroy(e);
    for (auto& set : p2p_ev)
      for (auto& e : set)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : tree_ev)
      if (e) (void)hipEventDestroy(e);
  }
}

}  // namespace hpm

using namespace hpm;

extern "C" {

const char* hpm_status_string(hpm_status s) {
  switch (s) {
    case HPM_OK: return "HPM_OK";
    case HPM_ERR_INVALID_ARG: return "HPM_ERR_INVALID_ARG";
    case HPM_ERR_OUT_OF_BOX: return "HPM_ERR_OUT_OF_BOX";
    case HPM_ERR_NONFINITE: return "HPM_ERR_NONFINITE";
    case HPM_ERR_NO_MEMORY: return "HPM_ERR_NO_MEMORY";
    case HPM_ERR_DEVICE: return "HPM_ERR_DEVICE";
    case HPM_ERR_UNSUPPORTED: return "HPM_ERR_UNSUPPORTED";
    case HPM_ERR_NOT_READY: return "HPM_ERR_NOT_READY";
  }
  return "HPM_ERR_UNKNOWN";
}

const char* hpm_last_error(void) { return g_last_error.c_str(); }

int32_t hpm_abi_version(void) { return HPM_ABI_VERSION; }

hpm_status hpm_plan_create(const hpm_problem* problem, int64_t n, const void* x, const void* y,
                           const void* z, void* stream, hpm_plan** out) {
  if (out) *out = nullptr;
  hpm_plan_s* pl = nullptr;
  hpm_status st = guarded([&] {
    if (!out) fail(HPM_ERR_INVALID_ARG, "out is NULL");
    check_problem(problem);
    check_size(problem, n);
    if (!x || !y || !z) fail(HPM_ERR_INVALID_ARG, "position pointer is NULL");
    pl = new hpm_plan_s();
    create_plan(pl->p, problem, n, x, y, z, (hipStream_t)stream);
  });
  if (st != HPM_OK) {
    delete pl;
    return st;
  }
  *out = pl;
  return HPM_OK;
}

hpm_status hpm_plan_execute(hpm_plan* plan, const void* m, void* phi, void* ax, void* ay,
                            void* az, void* stream) {
  return guarded([&] {
    if (!plan) fail(HPM_ERR_INVALID_ARG, "plan is NULL");
    if (!m || !phi || !ax || !ay || !az) fail(HPM_ERR_INVALID_ARG, "array pointer is NULL");
    if (!plan->p.valid) fail(HPM_ERR_INVALID_ARG, "plan has no valid tree (a rebuild failed)");
    execute_plan(plan->p, m, phi, ax, ay, az, (hipStream_t)stream);
  });
}

// routes a plan can evaluate with: its own; all three when it was made with the cell spectra and
// standard gridlets; with extended gridlets the cell route and (N_g = 4, 6) the padded grid
static bool route_allowed(const Plan& p, int32_t mode) {
  if (mode != HPM_M2L_GRID && mode != HPM_M2L_CELLS && mode != HPM_M2L_SHARED) return false;
  if (p.prob.m2l_mode == HPM_M2L_GRID) return mode == HPM_M2L_GRID;
  if (p.ext) return mode == HPM_M2L_CELLS || (mode == HPM_M2L_GRID && (p.ng == 4 || p.ng == 6));
  return true;
}

hpm_status hpm_plan_set_route(hpm_plan* plan, int32_t m2l_mode) {
  return guarded([&] {
    if (!plan) fail(HPM_ERR_INVALID_ARG, "plan is NULL");
    if (m2l_mode != HPM_M2L_GRID && m2l_mode != HPM_M2L_CELLS && m2l_mode != HPM_M2L_SHARED)
      fail(HPM_ERR_INVALID_ARG, "m2l_mode must be HPM_M2L_GRID, HPM_M2L_CELLS or HPM_M2L_SHARED");
    if (!route_allowed(plan->p, m2l_mode))
      fail(HPM_ERR_UNSUPPORTED, "the plan was not built for this source-to-target route");
    plan->p.route = m2l_mode;
  });
}

hpm_status hpm_plan_set_overlap(hpm_plan* plan, int32_t on) {
  return guarded([&] {
    if (!plan) fail(HPM_ERR_INVALID_ARG, "plan is NULL");
    if (on != 0 && on != 1) fail(HPM_ERR_INVALID_ARG, "on must be 0 or 1");
    plan->p.overlap = on != 0;
  });
}

hpm_status hpm_plan_set_fp32_strict(hpm_plan* plan, int32_t on) {
  return guarded([&] {
    if (!plan) fail(HPM_ERR_INVALID_ARG, "plan is NULL");
    if (on != 0 && on != 1) fail(HPM_ERR_INVALID_ARG, "on must be 0 or 1");
    const Plan& p = plan->p;
    if (on && (p.prec != HPM_F32 || (p.ng != 4 && p.ng != 6)))
      fail(HPM_ERR_UNSUPPORTED, "the all-FP32 source-to-target step is built for FP32 plans at "
                                "ng = 4 and 6");
    plan->p.fp32_strict = on != 0;
  });
}

hpm_status hpm_plan_autotune(hpm_plan* plan, const void* m, void* phi, void* ax, void* ay,
                             void* az, int32_t reps, void* stream, int32_t* mode, double* ms) {
  return guarded([&] {
    if (!plan) fail(HPM_ERR_INVALID_ARG, "plan is NULL");
    if (!m || !phi || !ax || !ay || !az) fail(HPM_ERR_INVALID_ARG, "array pointer is NULL");
    if (reps < 1 || reps > 1000) fail(HPM_ERR_INVALID_ARG, "reps must be 1..1000");
    Plan& p = plan->p;
    if (!p.valid) fail(HPM_ERR_INVALID_ARG, "plan has no valid tree (a rebuild failed)");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HPM_HIP(hipEventCreate(&e0));
    HPM_HIP(hipEventCreate(&e1));
    const int32_t first = p.route;
    int32_t best = first;
    double best_ms = -1.0;
    double per[3] = {-1.0, -1.0, -1.0};
    hpm_status st = guarded([&] {
      for (int32_t r = HPM_M2L_GRID; r <= HPM_M2L_SHARED; ++r) {
        if (!route_allowed(p, r)) continue;
        p.route = r;
        execute_plan(p, m, phi, ax, ay, az, s);  // untimed: first use of the route's kernels
        HPM_HIP(hipEventRecord(e0, s));
        for (int k = 0; k < reps; ++k) execute_plan(p, m, phi, ax, ay, az, s);
        HPM_HIP(hipEventRecord(e1, s));
        HPM_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        HPM_HIP(hipEventElapsedTime(&t, e0, e1));
        per[r] = double(t) / reps;
        if (best_ms < 0.0 || per[r] < best_ms) {
          best_ms = per[r];
          best = r;
        }
      }
    });
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != HPM_OK) {
      p.route = first;
      fail(st, hpm_last_error());
    }
    p.route = best;
    if (mode) *mode = best;
    if (ms)
      for (int r = 0; r < 3; ++r) ms[r] = per[r];
  });
}

hpm_status hpm_plan_rebuild(hpm_plan* plan, int64_t n, const void* x, const void* y,
                            const void* z, void* stream) {
  return guarded([&] {
    if (!plan) fail(HPM_ERR_INVALID_ARG, "plan is NULL");
    check_size(&plan->p.prob, n);
    if (!x || !y || !z) fail(HPM_ERR_INVALID_ARG, "position pointer is NULL");
    rebuild_plan(plan->p, n, x, y, z, (hipStream_t)stream);
  });
}

hpm_status hpm_plan_enable_timing(hpm_plan* plan, int32_t on) {
  return guarded([&] {
    if (!plan) fail(HPM_ERR_INVALID_ARG, "plan is NULL");
    Plan& p = plan->p;
    if (on && !p.events_created) {
      for (auto& set : p.ev)
        for (auto& e : set) HPM_HIP(hipEventCreate(&e));
      for (auto& set : p.p2p_ev)
        for (auto& e : set) HPM_HIP(hipEventCreate(&e));
      for (auto& e : p.tree_ev) HPM_HIP(hipEventCreate(&e));
      p.events_created = true;
    }
    while (p.ring_count > 0) drain_one(p);
    drain_tree(p);
    for (double& v : p.stage_ms) v = 0.0;
    p.n_exec = p.n_build = 0;
    p.timing = on != 0;
  });
}

hpm_status hpm_plan_stage_times(hpm_plan* plan, double* ms, int64_t* n_exec, int64_t* n_build) {
  return guarded([&] {
    if (!plan || !ms) fail(HPM_ERR_INVALID_ARG, "NULL argument");
    Plan& p = plan->p;
    while (p.ring_count > 0) drain_one(p);
    drain_tree(p);
    for (int k = 0; k <= Plan::kStages + 1; ++k) ms[k] = p.stage_ms[k];
    if (n_exec) *n_exec = p.n_exec;
    if (n_build) *n_build = p.n_build;
  });
}

void hpm_plan_destroy(hpm_plan* plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  delete plan;
}

hpm_status hpm_solve(const hpm_problem* problem, int64_t n, const void* x, const void* y,
                     const void* z, const void* m, void* phi, void* ax, void* ay, void* az,
                     void* stream) {
  hpm_plan* plan = nullptr;
  hpm_status st = hpm_plan_create(problem, n, x, y, z, stream, &plan);
  if (st != HPM_OK) return st;
  st = hpm_plan_execute(plan, m, phi, ax, ay, az, stream);
  if (st == HPM_OK)
    st = guarded([&] { HPM_HIP(hipStreamSynchronize((hipStream_t)stream)); });
  hpm_plan_destroy(plan);
  return st;
}

hpm_status hpm_plan_info_get(const hpm_plan* plan, hpm_plan_info* info) {
  return guarded([&] {
    if (!plan || !info) fail(HPM_ERR_INVALID_ARG, "NULL argument");
    const Plan& p = plan->p;
    *info = hpm_plan_info{};
    info->n_levels = p.nlevels;
    info->ng = p.ng;
    info->n_particles = p.n;
    info->n_cells = p.ncells;
    info->n_leaves = p.nleaves;
    info->n_targets = p.nlevels > 2 ? p.ncells - p.level_off[2] : 0;
    for (int l = 0; l < kMaxLevelsHost; ++l)
      info->cells_per_level[l] = (l < p.nlevels) ? p.level_off[l + 1] - p.level_off[l] : 0;
    long long pairs = 0;
    if (p.pairs.p) {  // counted on the device by the near-list build
      HPM_HIP(hipDeviceSynchronize());
      HPM_HIP(hipMemcpy(&pairs, p.pairs.p, sizeof(pairs), hipMemcpyDeviceToHost));
    }
    info->p2p_pairs = pairs;
    info->device_bytes = int64_t(p.device_bytes());
  });
}

hpm_status hpm_plan_copy_perm(const hpm_plan* plan, int32_t* perm) {
  return guarded([&] {
    if (!plan || !perm) fail(HPM_ERR_INVALID_ARG, "NULL argument");
    HPM_HIP(hipMemcpy(perm, plan->p.perm.p, size_t(plan->p.n) * 4, hipMemcpyDeviceToHost));
  });
}

static void level_range(const Plan& p, int32_t level, int* off, int* cnt) {
  if (level < 0 || level >= p.nlevels) fail(HPM_ERR_INVALID_ARG, "level has no cells");
  *off = p.level_off[level];
  *cnt = p.level_off[level + 1] - p.level_off[level];
}

hpm_status hpm_plan_copy_cells(const hpm_plan* plan, int32_t level, int32_t* coords, int32_t* pb,
                               int32_t* pe, int32_t* split, int32_t* parent) {
  return guarded([&] {
    if (!plan) fail(HPM_ERR_INVALID_ARG, "plan is NULL");
    const Plan& p = plan->p;
    int off, cnt;
    level_range(p, level, &off, &cnt);
    std::vector<int32_t> tmp(cnt);
    if (coords) {
      HPM_HIP(hipMemcpy(tmp.data(), p.ccoord.as<int>() + off, size_t(cnt) * 4, hipMemcpyDeviceToHost));
      for (int i = 0; i < cnt; ++i) {
        coords[3 * i] = tmp[i] & 1023;
        coords[3 * i + 1] = (tmp[i] >> 10) & 1023;
        coords[3 * i + 2] = (tmp[i] >> 20) & 1023;
      }
    }
    if (pb) HPM_HIP(hipMemcpy(pb, p.cpb.as<int>() + off, size_t(cnt) * 4, hipMemcpyDeviceToHost));
    if (pe) HPM_HIP(hipMemcpy(pe, p.cpe.as<int>() + off, size_t(cnt) * 4, hipMemcpyDeviceToHost));
    if (split) {
      HPM_HIP(hipMemcpy(split, p.cflags.as<int>() + off, size_t(cnt) * 4, hipMemcpyDeviceToHost));
      for (int i = 0; i < cnt; ++i) split[i] &= 1;
    }
    if (parent) {
      HPM_HIP(hipMemcpy(parent, p.cparent.as<int>() + off, size_t(cnt) * 4, hipMemcpyDeviceToHost));
      if (level > 0)
        for (int i = 0; i < cnt; ++i) parent[i] -= p.level_off[level - 1];
    }
  });
}

static hpm_status copy_rows(const hpm_plan* plan, int32_t level, void* host, bool locals) {
  return guarded([&] {
    if (!plan || !host) fail(HPM_ERR_INVALID_ARG, "NULL argument");
    const Plan& p = plan->p;
    if (level < 2) fail(HPM_ERR_INVALID_ARG, "gridlets exist at levels >= 2");
    int off, cnt;
    level_range(p, level, &off, &cnt);
    const DevBuf& b = locals ? p.local : p.gridlet;
    const size_t row = size_t(locals ? p.ML : p.M) * p.elem;
    HPM_HIP(hipMemcpy(host, static_cast<const char*>(b.p) + size_t(off) * row, size_t(cnt) * row,
                      hipMemcpyDeviceToHost));
  });
}

hpm_status hpm_plan_copy_gridlets(const hpm_plan* plan, int32_t level, void* host) {
  return copy_rows(plan, level, host, false);
}

hpm_status hpm_plan_copy_locals(const hpm_plan* plan, int32_t level, void* host) {
  return copy_rows(plan, level, host, true);
}

hpm_status hpm_plan_copy_local_offsets(const hpm_plan* plan, int32_t level, double* host) {
  return guarded([&] {
    if (!plan || !host) fail(HPM_ERR_INVALID_ARG, "NULL argument");
    const Plan& p = plan->p;
    if (level < 2) fail(HPM_ERR_INVALID_ARG, "local potentials exist at levels >= 2");
    int off, cnt;
    level_range(p, level, &off, &cnt);
    std::vector<char> c(size_t(cnt) * 2 * p.elem);
    HPM_HIP(hipMemcpy(c.data(), static_cast<const char*>(p.lofs.p) + size_t(off) * 2 * p.elem,
                      c.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < cnt; ++i) {
      if (p.prec == HPM_F32) {
        const float* ci = reinterpret_cast<const float*>(c.data()) + 2 * i;
        host[i] = double(ci[0]) + double(ci[1]);
      } else {
        const double* ci = reinterpret_cast<const double*>(c.data()) + 2 * i;
        host[i] = ci[0] + ci[1];
      }
    }
  });
}

hpm_status hpm_plan_bytes_estimate(const hpm_problem* problem, int64_t n, int64_t* bytes) {
  return guarded([&] {
    if (!bytes) fail(HPM_ERR_INVALID_ARG, "bytes is NULL");
    check_problem(problem);
    check_size(problem, n);
    *bytes = int64_t(plan_bytes_estimate(*problem, n));
  });
}

hpm_status hpm_direct_sum(int32_t precision, int64_t n, const void* x, const void* y,
                          const void* z, const void* m, int64_t n_targets, const int32_t* targets,
                          double gconst, double softening, int32_t kernel, double screening,
                          double* phi, double* ax, double* ay, double* az, void* stream) {
  return guarded([&] {
    if (precision != HPM_F32 && precision != HPM_F64) fail(HPM_ERR_INVALID_ARG, "bad precision");
    if (n < 1 || n > (int64_t(1) << 30) || n_targets < 0 || n_targets > n)
      fail(HPM_ERR_INVALID_ARG, "bad sizes");
    if (!x || !y || !z || !m || (n_targets > 0 && (!targets || !phi || !ax || !ay || !az)))
      fail(HPM_ERR_INVALID_ARG, "NULL pointer");
    if (!(softening >= 0.0) || !(gconst > 0.0)) fail(HPM_ERR_INVALID_ARG, "bad constants");
    check_kernel(kernel, screening);
    launch_direct_sum(precision, n, x, y, z, m, n_targets, targets, gconst, softening,
                      PairKernel{kernel, screening}, phi, ax, ay, az, (hipStream_t)stream);
  });
}

}  // extern "C"
