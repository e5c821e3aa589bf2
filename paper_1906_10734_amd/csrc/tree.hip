// Oct-tree construction on the device (Sec. 1): Morton keys, a stable LSD radix sort of
// (key, input index), levels of real cells by the split rule, child tables, the 27-cube
// neighbourhood of every cell, the leaf list, the virtual cubes of the interaction zones, and
// the list of split cells; about a dozen launches and one host synchronisation per build.
//
// Cells live in one id space with the levels contiguous and each level in Morton order. Every
// level is built at once from the sorted keys (see "Levels"). Neighbour entry encoding (27 per
// cell, x fastest):
//   >= 0        the real cell at that position (same level)
//   -1          no particle there, or outside the box
//   <= -2       the position lies inside the coarser leaf with id (-2 - entry); its particles are
//               the part of that leaf's range whose key prefix at this level matches the position
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "dev_common.h"
#include "hpm_internal.h"
#include "zones.h"

namespace hpm {

// ---------------------------------------------------------------------------------------------
// Workgroup scan
// ---------------------------------------------------------------------------------------------
// exclusive scan of one value per thread over a workgroup of NT threads, and the total
template <int NT>
__device__ __forceinline__ int group_scan(int v, int* s_w, int& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[wave] = x;
  __syncthreads();
  int pre = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wave) pre += s_w[w];
    all += s_w[w];
  }
  __syncthreads();
  total = all;
  return pre + x - v;
}

// ---------------------------------------------------------------------------------------------
// Stable LSD radix sort of (uint32 key, int32 value), 8 bits per pass, one launch per pass
// ---------------------------------------------------------------------------------------------
// The key kernel also counts every pass's digits over the whole input (the digit counts do not
// depend on the order), so a pass needs only the counts of the tiles before its own for each
// digit. A tile takes its index in the order workgroups start (an atomic counter), publishes its
// own digit counts, and walks back over the tiles before it, adding their counts until one has
// published its inclusive prefix; then it publishes its own inclusive prefix and scatters. Each
// status word holds a flag (2 bits: 1 counts, 2 inclusive prefix) and the value together, read
// and written as one 64-bit atomic, so no other ordering is needed. A tile waits only on tiles
// that started before it; should one not have published after a long wait, the waiting tile
// counts that tile's keys itself.
constexpr int kRsThreads = 256;
constexpr unsigned long long kRsFlagCount = 1ull << 62, kRsFlagPrefix = 2ull << 62;
constexpr unsigned long long kRsValue = (1ull << 62) - 1;
constexpr int kRsSpin = 1 << 14;
constexpr int kRsLook = 8;
constexpr int kRsMaxPasses = 4;

struct SortArgs {
  int n;
  int ntiles;
  int rounds;           // a tile is rounds * 256 consecutive items
  const uint32_t* kin;
  const int* vin;
  uint32_t* kout;
  int* vout;
  int shift;            // digit = (key >> shift) & 255
  int pass;
  unsigned long long* status;  // [passes][ntiles][256]
  int* tile_ctr;               // [kRsMaxPasses] next tile index of each pass
  const int* ghist;            // [kRsMaxPasses][256] digit counts of each pass
  // last pass: the positions, gathered into sorted order
  const void* x;
  const void* y;
  const void* z;
  void* xs;
  void* ys;
  void* zs;
};

template <typename T>
__global__ __launch_bounds__(256) void k_keys(int n, const T* x, const T* y, const T* z, double lo0,
                                              double lo1, double lo2, double hi0, double hi1,
                                              double hi2, double scale, int depth, int passes,
                                              uint32_t* keys, int* vals, int* box, int* ghist) {
  __shared__ int s_h[kRsMaxPasses][256];
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kRsMaxPasses; ++q) s_h[q][tid] = 0;
  __syncthreads();
  const int maxc = (1 << depth) - 1;
  for (int i = blockIdx.x * 256 + tid; i < n; i += gridDim.x * 256) {
    const double px = double(x[i]), py = double(y[i]), pz = double(z[i]);
    int bad = 0;
    if (!(isfinite(px) && isfinite(py) && isfinite(pz))) bad = 2;
    else if (!(px >= lo0 && px <= hi0 && py >= lo1 && py <= hi1 && pz >= lo2 && pz <= hi2)) bad = 1;
    uint32_t k = 0;
    if (bad) {
      box[bad == 2 ? Plan::kBoxNonfinite : Plan::kBoxOutOfBox] = 1;
    } else {
      // cube index floor((p - lo) * 2^D / size), clamped: the upper face belongs to the last cube
      const int ix = min(max(int(floor((px - lo0) * scale)), 0), maxc);
      const int iy = min(max(int(floor((py - lo1) * scale)), 0), maxc);
      const int iz = min(max(int(floor((pz - lo2) * scale)), 0), maxc);
      k = morton3(uint32_t(ix), uint32_t(iy), uint32_t(iz), depth);
    }
    keys[i] = k;
    vals[i] = i;
    for (int q = 0; q < passes; ++q) atomicAdd(&s_h[q][(k >> (8 * q)) & 255u], 1);
  }
  __syncthreads();
  for (int q = 0; q < passes; ++q)
    if (s_h[q][tid]) atomicAdd(&ghist[q * 256 + tid], s_h[q][tid]);
}

template <typename T, bool LAST>
__global__ __launch_bounds__(kRsThreads) void k_sort_pass(SortArgs a) {
  __shared__ int s_tile;
  __shared__ int s_cnt[256];
  __shared__ int run[256];
  __shared__ int wcnt[kRsThreads / 64][256];
  __shared__ int s_w[kRsThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(&a.tile_ctr[a.pass], 1);
  s_cnt[tid] = 0;
  __syncthreads();
  const int tile = s_tile;
  const int base = tile * a.rounds * kRsThreads;
  for (int r = 0; r < a.rounds; ++r) {
    const int i = base + r * kRsThreads + tid;
    if (i < a.n) atomicAdd(&s_cnt[(a.kin[i] >> a.shift) & 255u], 1);
  }
  __syncthreads();
  // thread d: the count of digit d in the tiles before this one
  const unsigned long long own = (unsigned long long)s_cnt[tid];
  unsigned long long* st = a.status + (size_t(a.pass) * a.ntiles) * 256;
  __hip_atomic_store(&st[size_t(tile) * 256 + tid], (tile == 0 ? kRsFlagPrefix : kRsFlagCount) | own,
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // the walk back reads kRsLook tiles' words at once (independent loads), nearest first
  unsigned long long excl = 0;
  bool done = tile == 0;
  for (int j0 = tile - 1; !done && j0 >= 0; j0 -= kRsLook) {
    unsigned long long win[kRsLook];
#pragma unroll
    for (int k = 0; k < kRsLook; ++k)
      win[k] = (j0 - k >= 0) ? __hip_atomic_load(&st[size_t(j0 - k) * 256 + tid], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                             : 0ull;
#pragma unroll
    for (int k = 0; k < kRsLook; ++k) {
      const int j = j0 - k;
      if (done || j < 0) continue;
      unsigned long long w = win[k];
      for (int spin = 0; !(w >> 62) && spin < kRsSpin; ++spin)
        w = __hip_atomic_load(&st[size_t(j) * 256 + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!(w >> 62)) {  // not published yet: count digit tid in tile j directly
        const int jb = j * a.rounds * kRsThreads, je = min(a.n, jb + a.rounds * kRsThreads);
        unsigned long long c = 0;
        for (int i = jb; i < je; ++i) c += ((a.kin[i] >> a.shift) & 255u) == uint32_t(tid);
        w = kRsFlagCount | c;
      }
      excl += w & kRsValue;
      if ((w >> 62) == 2) done = true;
    }
  }
  if (tile > 0)
    __hip_atomic_store(&st[size_t(tile) * 256 + tid], kRsFlagPrefix | (excl + own), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  // first output position of digit tid: items of smaller digits, then of earlier tiles
  int tot;
  const int dstart = group_scan<kRsThreads>(a.ghist[a.pass * 256 + tid], s_w, tot);
  run[tid] = dstart + int(excl);
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  // items in rounds of 256 in index order; within a round the rank of an item among equal digits
  // comes from wave ballots (lanes) and a per-digit prefix over the four waves: a stable order
  for (int r = 0; r < a.rounds; ++r) {
    const int i = base + r * kRsThreads + tid;
    const bool valid = i < a.n;
    uint32_t key = 0;
    int val = 0;
    if (valid) {
      key = a.kin[i];
      val = a.vin[i];
    }
    const uint32_t d = (key >> a.shift) & 255u;
#pragma unroll
    for (int w = 0; w < kRsThreads / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    uint64_t eq = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t mb = __ballot(valid && bit);
      eq &= bit ? mb : ~mb;
    }
    const int rank = __popcll(eq & lt);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(eq);
    __syncthreads();
    {
      int acc = run[tid];
#pragma unroll
      for (int w = 0; w < kRsThreads / 64; ++w) {
        const int c = wcnt[w][tid];
        wcnt[w][tid] = acc;
        acc += c;
      }
      run[tid] = acc;
    }
    __syncthreads();
    if (valid) {
      const int pos = wcnt[wave][d] + rank;
      if (pos >= 0 && pos < a.n) {  // always true for consistent counts
        a.kout[pos] = key;
        a.vout[pos] = val;
        if constexpr (LAST) {
          if (val >= 0 && val < a.n) {
            static_cast<T*>(a.xs)[pos] = static_cast<const T*>(a.x)[val];
            static_cast<T*>(a.ys)[pos] = static_cast<const T*>(a.y)[val];
            static_cast<T*>(a.zs)[pos] = static_cast<const T*>(a.z)[val];
          }
        }
      }
    }
    __syncthreads();
  }
}

// Tile size of the sort passes in rounds of 256 keys: 1024 keys up to 2^20 (at most 1024 tiles,
// all resident at once), larger tiles above, so that the walk back over tiles still running
// stays short.
static int sort_rounds(int n) { return n <= (1 << 20) ? 4 : (n <= (1 << 22) ? 16 : 64); }

// The sort state that the next build needs cleared (digit counts, tile counters, status words
// of the tiles used), cleared after this build's passes by the tree's count kernel.
struct SortClear {
  int* ghist;
  int* tile_ctr;
  unsigned long long* status;
  size_t status_words;
};

// Sorts the keys of k_keys (in tmp_keys, tmp_vals) into (keys, perm), gathering the positions
// into (xs, ys, zs) on the last pass.
template <typename T>
static void sort_and_gather(Plan& p, int nbits, const void* x, const void* y, const void* z,
                            hipStream_t s) {
  const int n = int(p.n);
  const int passes = (nbits + 7) / 8;
  SortArgs a;
  a.n = n;
  a.rounds = sort_rounds(n);
  a.ntiles = std::max(1, (n + a.rounds * kRsThreads - 1) / (a.rounds * kRsThreads));
  a.status = p.sort_status.as<unsigned long long>();
  a.tile_ctr = p.sort_ctr.as<int>();
  a.ghist = p.sort_ctr.as<int>() + kRsMaxPasses;
  a.x = x;
  a.y = y;
  a.z = z;
  a.xs = p.xs.p;
  a.ys = p.ys.p;
  a.zs = p.zs.p;
  uint32_t *ka = p.tmp_keys.as<uint32_t>(), *kb = p.keys.as<uint32_t>();
  int *va = p.tmp_vals.as<int>(), *vb = p.perm.as<int>();
  for (int q = 0; q < passes; ++q) {
    a.kin = ka;
    a.vin = va;
    a.kout = kb;
    a.vout = vb;
    a.shift = 8 * q;
    a.pass = q;
    if (q + 1 == passes) k_sort_pass<T, true><<<a.ntiles, kRsThreads, 0, s>>>(a);
    else k_sort_pass<T, false><<<a.ntiles, kRsThreads, 0, s>>>(a);
    HPM_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  // the sorted buffers are swapped in rather than copied
  if (ka != p.keys.as<uint32_t>()) {
    p.keys.swap(p.tmp_keys);
    p.perm.swap(p.tmp_vals);
  }
}


// ---------------------------------------------------------------------------------------------
// Levels
// ---------------------------------------------------------------------------------------------
// The cells follow from the sorted keys alone. A cell of level l is a run of equal level-l key
// prefixes whose parent run (level l - 1) was split, and a run is split when it holds more than
// leaf_capacity particles and l < D (uniform trees: when l < D). Particle counts only shrink
// from a run to its sub-runs, so the cells that contain particle i are its runs of levels
// 0 .. L(i), L(i) being the level of its leaf, and the cells that start at particle i are those
// of levels d(i) .. L(i), d(i) being the first level at which its key prefix differs from that of
// particle i - 1. A few launches build every level at once:
//   count: per workgroup of particles, the cells and leaves that start in it on each level;
//   scan:  one workgroup turns them into id bases (levels contiguous, each level in key order,
//          which is Morton order) and writes the level table;
//   emit:  the cells (key, coordinates, particle range, split flag), the leaf list and the list of
//          split cells;
//   hash:  cube id -> cell id;
//   link:  parent and child tables and the 27-cube neighbourhoods, by hash lookups.
// ---------------------------------------------------------------------------------------------
struct CellArrays {
  uint32_t* key;
  int* coord;
  int* pb;
  int* pe;
  int* parent;
  int* flags;
  int* child8;
  int* nbr27;
};

static CellArrays cells_of(Plan& p) {
  return {p.ckey.as<uint32_t>(), p.ccoord.as<int>(), p.cpb.as<int>(), p.cpe.as<int>(),
          p.cparent.as<int>(),   p.cflags.as<int>(),  p.child8.as<int>(), p.nbr27.as<int>()};
}

constexpr int kTreeThreads = 256;
constexpr int kTreeSeq = 2 * kMaxLevels;  // per workgroup: cells of each level, leaves of each
constexpr int kTreeMaxGroups = 16384;     // the count kernel's workgroups (rounds absorb the rest)

struct TreeArgs {
  const uint32_t* keys;  // sorted keys at depth D
  int n;
  int depth;
  int cap;
  int uniform;
  int rounds;           // particles per thread: workgroup b takes [b rounds 256, (b+1) rounds 256)
  int* blk;             // [workgroups][kTreeSeq]: counts, then id bases
  int* lev;             // level table
  int* box;             // mailbox words
  int* zero_words;      // cleared by the scan kernel for the later steps of the build (4 ints)
  unsigned long long* zero_pairs;  // near-zone pair count, likewise
  int* sort_ctr;                   // the sort's tile counters and digit counts (cleared)
  int sort_ctr_words;
  unsigned long long* sort_status; // the sort's status words (cleared)
  size_t sort_status_words;
  int64_t cap_cells;    // capacity of the cell arrays (emit and link do nothing above it)
  // emit / link
  CellArrays c;
  int* leaves;
  int* splits;          // cells with children of levels >= 1, in id order
  uint64_t* hslot;      // cube hash: (generation << 32 | cube id) per slot
  int* hval;            // cell id per slot
  uint32_t hmask;
  int hbits;
  uint32_t gen;         // this build's generation: slots of other generations are empty
};

// The sorted keys as a workgroup sees them: [lo, hi) staged in LDS, the rest in device memory.
struct KeyWin {
  const uint32_t* g;
  const uint32_t* s;
  int lo, hi;
  __device__ __forceinline__ uint32_t operator[](int j) const {
    return (j >= lo && j < hi) ? s[j - lo] : g[j];
  }
};
constexpr int kWinBefore = 128, kWinAfter = 384;  // around a round's 256 particles
constexpr int kWinKeys = kWinBefore + kTreeThreads + kWinAfter;

// stages the window of the round starting at particle base (all threads; ends with a barrier)
__device__ __forceinline__ KeyWin stage_window(const uint32_t* keys, int n, int base,
                                               uint32_t* s_keys) {
  KeyWin w{keys, s_keys, max(0, base - kWinBefore), min(n, base + kTreeThreads + kWinAfter)};
  for (int j = w.lo + int(threadIdx.x); j < w.hi; j += kTreeThreads) s_keys[j - w.lo] = keys[j];
  __syncthreads();
  return w;
}

// first index in [lo, hi) with keys[idx] >= v
__device__ __forceinline__ int lower_bound_win(const KeyWin& keys, int lo, int hi, uint32_t v) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (keys[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// first j in (i, hi] with keys[j] >= v (hi if none below hi); keys[i] < v
__device__ __forceinline__ int gallop_fwd(const KeyWin& keys, int i, int hi, uint32_t v) {
  int lo = i + 1, step = 1, j = i + 1;
  while (j < hi && keys[j] < v) {
    lo = j + 1;
    step <<= 1;
    j = i + step;
  }
  return lower_bound_win(keys, lo, min(j, hi), v);
}

// first j in [floor, i] with keys[j] >= v; keys[i] >= v and keys[floor] < v
__device__ __forceinline__ int gallop_back(const KeyWin& keys, int i, int floor, uint32_t v) {
  int hi = i, step = 1, j = i - 1;
  while (keys[j] >= v) {  // ends at floor at the latest
    hi = j;
    step <<= 1;
    j = max(i - step, floor);
  }
  return lower_bound_win(keys, j + 1, hi, v);
}

// First j in [lo, hi) with keys[j] >= v (hi if none) for every lane with `far`, the wave working
// on one lane's search at a time: a round probes 64 evenly spaced keys of the bracket and keeps
// the part between the last probe below v and the first at or above it, so a bracket of m keys
// takes about log_64 m rounds of parallel loads instead of 2 log_2 m dependent ones. Called by
// the whole wave; lanes without `far` get res back unchanged.
__device__ __forceinline__ int wave_lower_bound(const KeyWin& keys, bool far, int lo, int hi,
                                                uint32_t v, int res) {
  const int lane = threadIdx.x & 63;
  uint64_t pend = __ballot(far);
  while (pend) {
    const int src = __ffsll((unsigned long long)pend) - 1;
    pend &= pend - 1;
    int l = __shfl(lo, src, 64), h = __shfl(hi, src, 64);
    const uint32_t vv = uint32_t(__shfl(int(v), src, 64));
    // the answer lies in [l, h]: keys before l are below vv, and h is the bracket's end or holds
    // a key at or above vv
    while (h - l > 64) {
      const int step = (h - l + 63) >> 6;
      const int q = l + (lane + 1) * step - 1;
      const uint64_t m = __ballot(q < h && keys[q] >= vv);
      if (m) {
        const int f = __ffsll((unsigned long long)m) - 1;
        h = l + (f + 1) * step - 1;
        l += f * step;
      } else {
        l += ((h - l) / step) * step;  // past the last probe below h
      }
    }
    const int q = l + lane;
    const uint64_t m = __ballot(q < h && keys[q] >= vv);
    if (lane == src) res = m ? l + __ffsll((unsigned long long)m) - 1 : h;
  }
  return res;
}

// first j in (i, hi] with keys[j] >= v (hi if none below hi), keys[i] < v, for the lanes with
// `need` (i inside the window); whole wave
__device__ __forceinline__ int search_fwd(const KeyWin& kw, bool need, int i, int hi, uint32_t v) {
  int res = hi;
  bool far = false;
  const int wend = min(hi, kw.hi);
  if (need) {
    if (wend > i + 1 && kw[wend - 1] >= v) res = gallop_fwd(kw, i, wend - 1, v);
    else far = wend < hi;  // else every key below hi is below v
  }
  return wave_lower_bound(kw, far, wend, hi, v, res);
}

// first j in [0, i] with keys[j] >= v, keys[i] >= v, for the lanes with `need` (i inside the
// window); whole wave
__device__ __forceinline__ int search_back(const KeyWin& kw, bool need, int i, uint32_t v) {
  int res = 0;
  bool far = false;
  const int wbeg = kw.lo;
  if (need) {
    if (kw[wbeg] < v) res = gallop_back(kw, i, wbeg, v);
    else far = wbeg > 0;  // else the answer is 0
  }
  return wave_lower_bound(kw, far, 0, wbeg, v, res);
}

// The runs that start at one particle, walked level by level.
struct Walk {
  uint32_t key;
  int i;
  int lo;    // first level at which a cell starts here
  int end;   // end of the run of the previous level
  bool live; // cells start here at the levels still to come (until the leaf)
};

// whole wave (the searches are shared)
__device__ __forceinline__ Walk walk_init(const TreeArgs& a, const KeyWin& kw, int i) {
  Walk w{0u, i, kMaxLevels, 0, false};
  bool cand = i < a.n;
  int d = 0;
  if (cand) {
    w.key = kw[i];
    if (i > 0) {
      const uint32_t x = w.key ^ kw[i - 1];
      if (x == 0u) cand = false;  // same cube as the previous particle at every level
      else d = a.depth - (31 - __clz(int(x))) / 3;
    }
  }
  // the parent run (level d - 1) must be split: more than cap particles
  const bool check = cand && d >= 1 && !a.uniform;
  const int sh = check ? 3 * (a.depth - d + 1) : 0;
  const uint32_t pre = w.key >> sh;
  const int e = search_fwd(kw, check, i, a.n, (pre + 1u) << sh);
  const int b = search_back(kw, check, i, pre << sh);
  if (check && e - b <= a.cap) cand = false;
  if (cand) {
    w.lo = d;
    w.end = check ? e : a.n;
    w.live = true;
  }
  return w;
}

// level l of the walk (called for l = 0, 1, ... in order by the whole wave): a cell starts here
// (cell), it is a leaf (leaf), with cnt particles
__device__ __forceinline__ void walk_step(const TreeArgs& a, const KeyWin& kw, Walk& w, int l,
                                          bool& cell, bool& leaf, int& cnt) {
  cell = leaf = false;
  cnt = 0;
  const bool act = w.live && l >= w.lo;
  const int sh = 3 * (a.depth - l);
  const int e = search_fwd(kw, act && l > 0, w.i, w.end, ((w.key >> sh) + 1u) << sh);
  if (!act) return;
  cnt = (l == 0 ? a.n : e) - w.i;
  cell = true;
  leaf = a.uniform ? (l >= a.depth) : (cnt <= a.cap || l >= a.depth);
  w.end = w.i + cnt;
  if (leaf) w.live = false;
}

__global__ __launch_bounds__(kTreeThreads) void k_tree_count(TreeArgs a) {
  __shared__ int s_cnt[kTreeSeq];
  __shared__ uint32_t s_keys[kWinKeys];
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < kTreeSeq) s_cnt[tid] = 0;
  // the sort that ran before is done with its state: clear it for the next build
  for (size_t w = size_t(blockIdx.x) * kTreeThreads + tid; w < a.sort_status_words;
       w += size_t(gridDim.x) * kTreeThreads)
    a.sort_status[w] = 0ull;
  if (blockIdx.x == 0)
    for (int w = tid; w < a.sort_ctr_words; w += kTreeThreads) a.sort_ctr[w] = 0;
  __syncthreads();
  for (int r = 0; r < a.rounds; ++r) {
    const int base = (blockIdx.x * a.rounds + r) * kTreeThreads, i = base + tid;
    const KeyWin kw = stage_window(a.keys, a.n, base, s_keys);
    Walk w = walk_init(a, kw, i);
    for (int l = 0; l < kMaxLevels; ++l) {
      bool cell, leaf;
      int cnt;
      walk_step(a, kw, w, l, cell, leaf, cnt);
      const uint64_t mc = __ballot(cell), ml = __ballot(leaf);
      if (lane == 0 && mc) atomicAdd(&s_cnt[l], __popcll(mc));
      if (lane == 0 && ml) atomicAdd(&s_cnt[kMaxLevels + l], __popcll(ml));
    }
    __syncthreads();  // the window is read before the next round stages its own
  }
  __syncthreads();
  if (tid < kTreeSeq) a.blk[size_t(blockIdx.x) * kTreeSeq + tid] = s_cnt[tid];
}

// One workgroup: the id bases of every count workgroup within each level (one wave scans a
// sequence over the workgroups in chunks of 64; the emit kernel adds the level's offset), the
// level table (levels contiguous, level-major), its copy in the mailbox, and the words the later
// launches of the build accumulate into, cleared.
constexpr int kTreeScanThreads = 1024;
__global__ __launch_bounds__(kTreeScanThreads) void k_tree_scan(TreeArgs a, int nb) {
  __shared__ int s_tot[kTreeSeq];
  __shared__ int s_off[kTreeSeq];
  __shared__ int s_lev[kLevWords];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int q = wave; q < kTreeSeq; q += kTreeScanThreads / 64) {
    int run = 0;
    for (int c0 = 0; c0 < nb; c0 += 16 * 64) {  // sixteen chunks of 64 read at once
      int v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int b = c0 + 64 * u + lane;
        v[u] = b < nb ? a.blk[size_t(b) * kTreeSeq + q] : 0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int b = c0 + 64 * u + lane;
        int x = v[u];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(x, o, 64);
          if (lane >= o) x += y;
        }
        if (b < nb) a.blk[size_t(b) * kTreeSeq + q] = run + x - v[u];  // within the level
        run += __shfl(x, 63, 64);
      }
    }
    if (lane == 0) s_tot[q] = run;
  }
  __syncthreads();
  if (tid == 0) {
    int oc = 0, ol = 0;
    for (int l = 0; l < kMaxLevels; ++l) {
      s_off[l] = oc;
      s_off[kMaxLevels + l] = ol;
      oc += s_tot[l];
      ol += s_tot[kMaxLevels + l];
    }
    for (int w = 0; w < kLevWords; ++w) s_lev[w] = 0;
    for (int l = 0; l < 16; ++l) {
      s_lev[kLevOff + l] = l < kMaxLevels ? s_off[l] : oc;
      s_lev[kLevCnt + l] = l < kMaxLevels ? s_tot[l] : 0;
    }
    s_lev[kLevCells] = oc;
    s_lev[kLevLeaves] = ol;
    s_lev[kLevLeavesLt2] = s_tot[kMaxLevels] + s_tot[kMaxLevels + 1];
    int ps = 0;
    for (int l = 0; l < 12; ++l) {
      s_lev[kLevLeafOff + l] = l < kMaxLevels ? s_off[kMaxLevels + l] : ol;
      s_lev[kLevSplitOff + l] = ps;  // split cells of levels 1 .. l-1
      if (l >= 1 && l < kMaxLevels) ps += s_tot[l] - s_tot[kMaxLevels + l];
    }
  }
  __syncthreads();
  if (tid < kLevWords) {
    a.lev[tid] = s_lev[tid];
    a.box[Plan::kBoxLev + tid] = s_lev[tid];
  }
  if (tid >= 64 && tid < 64 + 12) {  // split-list bounds of levels 1 .. L-1
    const int l = tid - 64;
    if (l >= 1 && s_lev[kLevCnt + l] > 0) a.box[Plan::kBoxCellLevels + l] = s_lev[kLevSplitOff + l];
  }
  if (tid == 128) {
    a.box[Plan::kBoxLeaves] = s_lev[kLevLeaves];
    a.box[Plan::kBoxLeavesLt2] = s_lev[kLevLeavesLt2];
    for (int w = 0; w < 4; ++w) a.zero_words[w] = 0;
    *a.zero_pairs = 0ull;
  }
}

// multiplicative (Fibonacci) hashing: the top "bits" bits of id times 2^32 / golden ratio
__device__ __forceinline__ uint32_t cube_hash(uint32_t id, int bits) {
  return (id * 0x9E3779B1u) >> (32 - bits);
}

__device__ __forceinline__ void chash_insert(const TreeArgs& a, uint32_t id, int v) {
  const uint64_t mine = (uint64_t(a.gen) << 32) | id;
  uint32_t h = cube_hash(id, a.hbits);
  for (uint32_t probe = 0; probe <= a.hmask;) {
    const uint64_t cur = __hip_atomic_load(&a.hslot[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (uint32_t(cur >> 32) == a.gen) {  // taken in this build
      h = (h + 1) & a.hmask;
      ++probe;
      continue;
    }
    if (atomicCAS(reinterpret_cast<unsigned long long*>(&a.hslot[h]), (unsigned long long)cur,
                  (unsigned long long)mine) == cur) {
      a.hval[h] = v;
      return;
    }
    // another insertion of this build took the slot first: look at it again
  }
}

__device__ __forceinline__ int chash_find(const TreeArgs& a, uint32_t id) {
  uint32_t h = cube_hash(id, a.hbits);
  for (uint32_t probe = 0; probe <= a.hmask; ++probe) {
    const uint64_t s = a.hslot[h];
    if (uint32_t(s >> 32) != a.gen) return -1;
    if (uint32_t(s) == id) return a.hval[h];
    h = (h + 1) & a.hmask;
  }
  return -1;
}

__global__ __launch_bounds__(kTreeThreads) void k_tree_emit(TreeArgs a) {
  __shared__ int s_run[kTreeSeq];
  __shared__ int s_w[2][kTreeThreads / 64];
  __shared__ int s_lev[kLevWords];
  __shared__ uint32_t s_keys[kWinKeys];
  if (int64_t(a.lev[kLevCells]) > a.cap_cells) return;  // the host grows the arrays and re-runs
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // this workgroup's first id on each level: its base within the level plus the level's offset
  if (tid < kTreeSeq)
    s_run[tid] = a.blk[size_t(blockIdx.x) * kTreeSeq + tid] +
                 a.lev[tid < kMaxLevels ? kLevOff + tid : kLevLeafOff + tid - kMaxLevels];
  if (tid < kLevWords) s_lev[tid] = a.lev[tid];
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  __syncthreads();
  for (int r = 0; r < a.rounds; ++r) {
    const int base = (blockIdx.x * a.rounds + r) * kTreeThreads, i = base + tid;
    const KeyWin kw = stage_window(a.keys, a.n, base, s_keys);
    Walk w = walk_init(a, kw, i);
    for (int l = 0; l < kMaxLevels; ++l) {
      bool cell, leaf;
      int cnt;
      walk_step(a, kw, w, l, cell, leaf, cnt);
      const uint64_t mc = __ballot(cell), ml = __ballot(leaf);
      if (lane == 0) {
        s_w[0][wave] = __popcll(mc);
        s_w[1][wave] = __popcll(ml);
      }
      __syncthreads();
      int pc = s_run[l], pl = s_run[kMaxLevels + l], tc = 0, tl = 0;
#pragma unroll
      for (int q = 0; q < kTreeThreads / 64; ++q) {
        if (q < wave) {
          pc += s_w[0][q];
          pl += s_w[1][q];
        }
        tc += s_w[0][q];
        tl += s_w[1][q];
      }
      if (cell) {
        const int id = pc + __popcll(mc & lt);
        const int sh = 3 * (a.depth - l);
        const uint32_t key = w.key >> sh;
        int x = 0, y = 0, z = 0;
        for (int b = 0; b < l; ++b) {
          x |= int((key >> (3 * b)) & 1u) << b;
          y |= int((key >> (3 * b + 1)) & 1u) << b;
          z |= int((key >> (3 * b + 2)) & 1u) << b;
        }
        a.c.key[id] = key;
        a.c.coord[id] = pack_coord(x, y, z);
        a.c.pb[id] = w.i;
        a.c.pe[id] = w.i + cnt;
        a.c.flags[id] = leaf ? 0 : 1;
        int4* ch = reinterpret_cast<int4*>(a.c.child8 + size_t(id) * 8);
        ch[0] = make_int4(-1, -1, -1, -1);
        ch[1] = make_int4(-1, -1, -1, -1);
        const int lrank = pl + __popcll(ml & lt);  // leaves before this cell in id order
        if (leaf) a.leaves[lrank] = id;
        else if (l >= 1)
          a.splits[s_lev[kLevSplitOff + l] + (id - s_lev[kLevOff + l]) -
                   (lrank - s_lev[kLevLeafOff + l])] = id;
      }
      __syncthreads();  // every thread has read s_run and s_w
      if (tid == 0) {
        s_run[l] += tc;
        s_run[kMaxLevels + l] += tl;
      }
      __syncthreads();
    }
  }
}

// thread per cell: its cube id -> cell id into the hash (a launch of its own, so that the emit
// kernel's level loop does not wait on the atomics)
__global__ __launch_bounds__(256) void k_tree_hash(TreeArgs a) {
  __shared__ int s_off[kMaxLevels + 1];
  const int ncells = a.lev[kLevCells];
  if (int64_t(ncells) > a.cap_cells) return;
  if (threadIdx.x <= kMaxLevels) s_off[threadIdx.x] = a.lev[kLevOff + threadIdx.x];
  __syncthreads();
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ncells; g += gridDim.x * blockDim.x)
    chash_insert(a, cube_id(level_of(g, s_off, kMaxLevels), a.c.key[g]), g);
}

// thread per (cell, neighbour entry): the neighbour entry of the 27-cube neighbourhood (x
// fastest); entry 13 also links the cell to its parent. The entry of position q on level l is
// the cell there, or else the deepest cell that contains q: -2 - id if that is a leaf (q lies
// inside it), -1 if it has children (the level-l cube at q is empty), and -1 outside the box.
__global__ __launch_bounds__(256) void k_tree_link(TreeArgs a) {
  __shared__ int s_off[kMaxLevels + 1];
  const int ncells = a.lev[kLevCells];
  if (int64_t(ncells) > a.cap_cells) return;
  if (threadIdx.x <= kMaxLevels) s_off[threadIdx.x] = a.lev[kLevOff + threadIdx.x];
  __syncthreads();
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < int64_t(ncells) * 27;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int g = int(t / 27), j = int(t % 27);
    const int l = level_of(g, s_off, kMaxLevels);
    const uint32_t key = a.c.key[g];
    int v = -1;
    if (j == 13) {
      v = g;
      int par = -1;
      if (l > 0) {
        par = chash_find(a, cube_id(l - 1, key >> 3));
        if (par >= 0) a.c.child8[size_t(par) * 8 + (key & 7u)] = g;
      }
      a.c.parent[g] = par;
    } else {
      const int pc = a.c.coord[g];
      const int qx = coord_x(pc) + j % 3 - 1, qy = coord_y(pc) + (j / 3) % 3 - 1,
                qz = coord_z(pc) + j / 9 - 1;
      const int side = 1 << l;
      if (qx >= 0 && qy >= 0 && qz >= 0 && qx < side && qy < side && qz < side) {
        const uint32_t q = morton3(uint32_t(qx), uint32_t(qy), uint32_t(qz), l);
        for (int k = l; k >= 0; --k) {
          const int id = chash_find(a, cube_id(k, q >> (3 * (l - k))));
          if (id < 0) continue;
          v = (k == l) ? id : ((a.c.flags[id] & 1) ? -1 : -2 - id);
          break;
        }
      }
    }
    a.c.nbr27[size_t(g) * 27 + j] = v;
  }
}

static void ensure_cells(Plan& p, int64_t need, int64_t keep, hipStream_t s) {
  if (need <= p.cap_cells) return;
  int64_t cap = std::max<int64_t>(need, p.cap_cells + p.cap_cells / 2);
  const size_t c4 = size_t(cap) * 4, k4 = size_t(keep) * 4;
  p.ckey.grow(c4, k4, s);
  p.ccoord.grow(c4, k4, s);
  p.cpb.grow(c4, k4, s);
  p.cpe.grow(c4, k4, s);
  p.cparent.grow(c4, k4, s);
  p.cflags.grow(c4, k4, s);
  p.child8.grow(c4 * 8, k4 * 8, s);
  p.nbr27.grow(c4 * 27, k4 * 27, s);
  p.cap_cells = cap;
}

// (re)allocates b and clears it when the allocation changes; true if it did
static bool reserve_cleared(DevBuf& b, size_t bytes, hipStream_t s) {
  if (bytes <= b.bytes && b.p) return false;
  b.reserve(bytes);
  HPM_HIP(hipMemsetAsync(b.p, 0, b.bytes, s));
  return true;
}

// the cube hash for the cell arrays' capacity (at least twice as many slots)
static void reserve_cube_hash(Plan& p, hipStream_t s) {
  int bits = 12;
  while ((int64_t(1) << bits) < 2 * p.cap_cells && bits < 31) ++bits;
  if (bits > p.chash_bits || !p.chash_slot.p) {
    p.chash_bits = std::max(bits, p.chash_bits);
    const size_t slots = size_t(1) << p.chash_bits;
    p.chash_slot.release();
    reserve_cleared(p.chash_slot, slots * 8, s);
    p.chash_val.reserve(slots * 4);
  }
}

static inline int nblk(int64_t n, int t) { return int((n + t - 1) / t); }

static void reserve_virt_set(Plan& p, int min_bits, hipStream_t s);
static void enqueue_virt_insert(Plan& p, hipStream_t s);

void build_tree(Plan& p, const void* x, const void* y, const void* z, hipStream_t s) {
  const hpm_problem& pr = p.prob;
  const int n = int(p.n);
  const bool uniform = pr.uniform_depth > 0;
  const int D = uniform ? pr.uniform_depth : pr.max_depth;
  p.depth = D;
  p.keys.reserve(size_t(n) * 4);
  p.perm.reserve(size_t(n) * 4);
  p.tmp_keys.reserve(size_t(n) * 4);
  p.tmp_vals.reserve(size_t(n) * 4);
  clear_box(p, Plan::kBoxOutOfBox, 2, s);

  p.xs.reserve(size_t(n) * p.elem);
  p.ys.reserve(size_t(n) * p.elem);
  p.zs.reserve(size_t(n) * p.elem);
  p.ms.reserve(size_t(n) * p.elem);
  // sort state: digit counts and tile counters, and the tiles' status words; all zero between
  // builds (cleared by the count kernel after the passes; cleared here if a build stopped short)
  const int passes = (3 * D + 7) / 8;
  const int rounds = sort_rounds(n);
  const int ntiles = std::max(1, nblk(n, rounds * kRsThreads));
  const size_t status_words = size_t(passes) * ntiles * 256;
  bool fresh = reserve_cleared(p.sort_ctr, size_t(kRsMaxPasses) * 257 * 4, s);
  fresh = reserve_cleared(p.sort_status, status_words * 8, s) || fresh;
  if (!p.sort_clean && !fresh) {
    HPM_HIP(hipMemsetAsync(p.sort_ctr.p, 0, p.sort_ctr.bytes, s));
    HPM_HIP(hipMemsetAsync(p.sort_status.p, 0, p.sort_status.bytes, s));
  }
  p.sort_clean = false;

  const double scale = double(1 << D) / pr.box_size;
  const double hi0 = pr.box_lo[0] + pr.box_size, hi1 = pr.box_lo[1] + pr.box_size,
               hi2 = pr.box_lo[2] + pr.box_size;
  int* ghist = p.sort_ctr.as<int>() + kRsMaxPasses;
  const int kgrid = std::max(1, std::min(nblk(n, 1024), 1024));  // about 4 keys per thread
  if (p.prec == HPM_F32) {
    k_keys<float><<<kgrid, 256, 0, s>>>(n, (const float*)x, (const float*)y, (const float*)z,
                                        pr.box_lo[0], pr.box_lo[1], pr.box_lo[2], hi0, hi1, hi2,
                                        scale, D, passes, p.tmp_keys.as<uint32_t>(),
                                        p.tmp_vals.as<int>(), p.dbox, ghist);
    HPM_LAUNCH_CHECK();
    sort_and_gather<float>(p, 3 * D, x, y, z, s);
  } else {
    k_keys<double><<<kgrid, 256, 0, s>>>(n, (const double*)x, (const double*)y, (const double*)z,
                                         pr.box_lo[0], pr.box_lo[1], pr.box_lo[2], hi0, hi1, hi2,
                                         scale, D, passes, p.tmp_keys.as<uint32_t>(),
                                         p.tmp_vals.as<int>(), p.dbox, ghist);
    HPM_LAUNCH_CHECK();
    sort_and_gather<double>(p, 3 * D, x, y, z, s);
  }
  // invalid positions got key 0, so the build below stays well defined; the flags are checked
  // at the synchronisation after the levels

  // capacity of the cell arrays: the cells a tree of this kind usually has (grown and the emit
  // and link launches repeated when the count says more)
  int64_t est = 64;
  if (uniform) {
    int64_t lvl = 1;
    est = 0;
    for (int l = 0; l <= D; ++l) {
      est += std::min<int64_t>(lvl, n);
      lvl *= 8;
    }
  } else {
    est = std::max<int64_t>(1024, 6 * int64_t(n) / std::max(1, pr.leaf_capacity) + 64);
  }
  ensure_cells(p, est, 0, s);

  TreeArgs a;
  a.keys = p.keys.as<uint32_t>();
  a.n = n;
  a.depth = D;
  a.cap = pr.leaf_capacity;
  a.uniform = uniform ? 1 : 0;
  a.rounds = std::max(1, nblk(nblk(n, kTreeThreads), kTreeMaxGroups));
  const int groups = std::max(1, nblk(n, kTreeThreads * a.rounds));
  p.tree_blk.reserve(size_t(groups) * kTreeSeq * 4);
  p.dlev.reserve(kLevWords * sizeof(int));
  a.blk = p.tree_blk.as<int>();
  a.lev = p.dlev.as<int>();
  a.box = p.dbox;
  p.vcount.reserve(4 * sizeof(int));  // cleared by the scan kernel
  p.pairs.reserve(16);
  a.zero_words = p.vcount.as<int>();
  a.zero_pairs = p.pairs.as<unsigned long long>();
  a.sort_ctr = p.sort_ctr.as<int>();
  a.sort_ctr_words = kRsMaxPasses * 257;
  a.sort_status = p.sort_status.as<unsigned long long>();
  a.sort_status_words = status_words;
  k_tree_count<<<groups, kTreeThreads, 0, s>>>(a);
  HPM_LAUNCH_CHECK();
  k_tree_scan<<<1, kTreeScanThreads, 0, s>>>(a, groups);
  HPM_LAUNCH_CHECK();
  p.sort_clean = true;
  const int* hl = p.hbox + Plan::kBoxLev;
  for (int attempt = 0;; ++attempt) {
    reserve_cube_hash(p, s);
    p.leaves.reserve(size_t(p.cap_cells) * 4);      // at most one leaf per cell
    p.cell_plist.reserve(size_t(p.cap_cells) * 4);  // and one split cell
    p.tree_gen = (p.tree_gen + 1u) ? p.tree_gen + 1u : 1u;  // 0 never names a build
    a.cap_cells = p.cap_cells;
    a.c = cells_of(p);
    a.leaves = p.leaves.as<int>();
    a.splits = p.cell_plist.as<int>();
    a.hslot = p.chash_slot.as<uint64_t>();
    a.hval = p.chash_val.as<int>();
    a.hbits = p.chash_bits;
    a.hmask = uint32_t((size_t(1) << p.chash_bits) - 1);
    a.gen = p.tree_gen;
    k_tree_emit<<<groups, kTreeThreads, 0, s>>>(a);
    HPM_LAUNCH_CHECK();
    k_tree_hash<<<std::max(1, std::min(nblk(p.cap_cells, 256), 4096)), 256, 0, s>>>(a);
    HPM_LAUNCH_CHECK();
    k_tree_link<<<std::max(1, std::min(nblk(p.cap_cells * 27, 256), 8192)), 256, 0, s>>>(a);
    HPM_LAUNCH_CHECK();
    if (!uniform) {
      reserve_virt_set(p, 0, s);
      enqueue_virt_insert(p, s);
    }
    enqueue_near_lists(p, s);
    sync_box(p, s);
    if (attempt == 0) {
      if (p.hbox[Plan::kBoxNonfinite]) fail(HPM_ERR_NONFINITE, "a particle position is not finite");
      if (p.hbox[Plan::kBoxOutOfBox])
        fail(HPM_ERR_OUT_OF_BOX, "a particle position is outside the box");
    }
    const int64_t total = hl[kLevCells];
    if (total <= p.cap_cells) break;
    if (attempt > 0) fail(HPM_ERR_DEVICE, "tree build: cell count changed between launches");
    // every launch after the count returned at once: grow and run them again
    ensure_cells(p, total + total / 4 + 64, 0, s);
  }
  // a virtual-cube set that filled up: a larger one, listed again
  while (!uniform && p.hbox[Plan::kBoxVirtFull]) {
    if (p.vhash_bits >= 30) fail(HPM_ERR_NO_MEMORY, "too many virtual cubes");
    reserve_virt_set(p, p.vhash_bits + 2, s);
    HPM_HIP(hipMemsetAsync(p.vcount.p, 0, 2 * sizeof(int), s));
    enqueue_virt_insert(p, s);
    enqueue_near_lists(p, s);  // (copies the two words to the mailbox)
    sync_box(p, s);
  }
  p.nlevels = 0;
  for (int l = 0; l <= D; ++l) {
    if (hl[kLevCnt + l] <= 0) break;
    p.level_off[l] = hl[kLevOff + l];
    p.nlevels = l + 1;
  }
  p.ncells = hl[kLevCells];
  for (int l = p.nlevels; l <= kMaxLevelsHost; ++l) p.level_off[l] = int(p.ncells);
  p.nleaves = p.hbox[Plan::kBoxLeaves];
  p.nleaves_lt2 = (p.nlevels > 2) ? p.hbox[Plan::kBoxLeavesLt2] : p.nleaves;
  p.nvirt = uniform ? 0 : p.hbox[Plan::kBoxVirt];
  p.n_items = p.hbox[Plan::kBoxTotal];
}



// ---------------------------------------------------------------------------------------------
// Virtual cubes: interaction-zone cube positions that are not cells of the tree but hold
// particles of a coarser leaf. Each is listed once (a hash set of cube ids, filled by every
// parent block that sees one) and appended to the cell arrays at ids ncells + v with its
// coordinates and particle range, so that its effective masses are fitted once per solve like a
// leaf's and the source-to-target kernels read them like any gridlet. The index v of a cube is
// the order in which it was first found; nothing computed from it depends on that order.
// ---------------------------------------------------------------------------------------------
struct VirtArgs {
  int depth;
  const int* lev;        // the tree's level table
  int64_t cap_cells;     // nothing to do while the cells outgrow the arrays
  const int* coord;
  const int* parent;
  const int* flags;
  const int* child8;
  const int* nbr27;
  const int* pb;
  const int* pe;
  const uint32_t* keys;  // sorted particle keys at depth D
  uint64_t* hslot;       // hash set: (generation << 32 | cube id) per slot
  int* hval;             // hash set: v per slot
  uint32_t mask;         // slots - 1
  int bits;              // slots = 2^bits
  uint32_t gen;
  int* count;            // [0] cubes listed, [1] the set is full
  int* vcubes;           // [v][3]: cube id, first and end sorted particle
  int* box;
};

// parents of targets: the cells of levels 1 .. L-2, [first, end) in id order
__device__ __forceinline__ void parent_range(const int* lev, int& first, int& end) {
  int nlev = 0;
  for (int l = 0; l < kMaxLevels; ++l)
    if (lev[kLevCnt + l] > 0) nlev = l + 1;
  first = lev[kLevOff + 1];
  end = nlev > 2 ? lev[kLevOff + nlev - 1] : first;
}

// One workgroup per parent of targets (grid-stride), one thread per slot of its 6^3 block: a
// nonempty virtual cube in the interaction zone of some child (every block cube except the 8
// children's own positions) joins the set; the thread that adds a new id takes the next index v
// and records the id and the cube's particle range at vcubes[v]. A full set raises count[1]. (The near-zone list launch that
// follows copies both words to the mailbox.)
__global__ __launch_bounds__(256) void k_virt_insert(VirtArgs a) {
  __shared__ int s_off[kMaxLevels + 1];
  const int tid = threadIdx.x;
  if (int64_t(a.lev[kLevCells]) > a.cap_cells) return;
  if (tid <= kMaxLevels) s_off[tid] = a.lev[kLevOff + tid];
  __syncthreads();
  int first, end;
  parent_range(a.lev, first, end);
  for (int par = first + blockIdx.x; par < end; par += gridDim.x) {
    if (tid >= 216 || !(a.flags[par] & 1)) continue;
    const int l = level_of(par, s_off, kMaxLevels) + 1;  // level of the block's cubes
    const int bx = tid % 6, by = (tid / 6) % 6, bz = tid / 36;
    if (bx >= 2 && bx <= 3 && by >= 2 && by <= 3 && bz >= 2 && bz <= 3) continue;  // children
    const int pc = a.coord[par];
    const IzSlot z = block_cube(coord_x(pc), coord_y(pc), coord_z(pc), l, par, tid, a.nbr27,
                                a.flags, a.child8);
    if (z.coarse < 0) continue;
    const int shift = 3 * (a.depth - l);
    const int cb = a.pb[z.coarse], ce = a.pe[z.coarse];
    int vb, ve;
    key_range_u32(a.keys, cb, ce, z.key << shift, (z.key + 1u) << shift, vb, ve);
    if (ve <= vb) continue;
    const uint32_t id = cube_id(l, z.key);
    const uint64_t mine = (uint64_t(a.gen) << 32) | id;
    uint32_t h = cube_hash(id, a.bits);
    bool placed = false;
    for (uint32_t probe = 0; probe <= a.mask;) {
      const uint64_t cur = __hip_atomic_load(&a.hslot[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (uint32_t(cur >> 32) == a.gen) {
        if (uint32_t(cur) == id) {  // listed already
          placed = true;
          break;
        }
        h = (h + 1) & a.mask;
        ++probe;
        continue;
      }
      if (atomicCAS(reinterpret_cast<unsigned long long*>(&a.hslot[h]), (unsigned long long)cur,
                    (unsigned long long)mine) == cur) {
        const int v = atomicAdd(&a.count[0], 1);
        a.hval[h] = v;
        a.vcubes[3 * v] = int(id);
        a.vcubes[3 * v + 1] = vb;
        a.vcubes[3 * v + 2] = ve;
        placed = true;
        break;
      }
      // the slot changed under us (another insertion of this build): look at it again
    }
    if (!placed) atomicExch(&a.count[1], 1);
  }
}

// Workgroups [0, nt): the source gridlet id of every slot of the 6^3 block of each parent of
// targets: a real cell id, ncells + v for virtual cube v (found in the hash set), or -1 (empty
// position, outside the box, or not a parent). Workgroups from nt on: coordinates, particle range
// and level of virtual cube v, stored at cell id ncells + v.
__global__ __launch_bounds__(256) void k_virt_finish(VirtArgs a, int first, int nt, int ncells,
                                                     int nvirt, int* table, int* coord, int* pb,
                                                     int* pe, int* vlevel, int* vlist) {
  __shared__ int s_off[kMaxLevels + 1];
  const int tid = threadIdx.x;
  if (int(blockIdx.x) >= nt) {
    const int v = (blockIdx.x - nt) * 256 + tid;
    if (v >= nvirt) return;
    const uint32_t id = uint32_t(a.vcubes[3 * v]);
    const int l = cube_id_level(id);
    const uint32_t key = id ^ (1u << (3 * l));
    int x = 0, y = 0, z = 0;
    for (int b = 0; b < l; ++b) {
      x |= int((key >> (3 * b)) & 1u) << b;
      y |= int((key >> (3 * b + 1)) & 1u) << b;
      z |= int((key >> (3 * b + 2)) & 1u) << b;
    }
    coord[ncells + v] = pack_coord(x, y, z);
    pb[ncells + v] = a.vcubes[3 * v + 1];
    pe[ncells + v] = a.vcubes[3 * v + 2];
    vlevel[v] = l;
    vlist[v] = ncells + v;
    return;
  }
  if (tid <= kMaxLevels) s_off[tid] = a.lev[kLevOff + tid];
  __syncthreads();
  if (tid >= 216) return;
  const int par = first + blockIdx.x;
  int src = -1;
  if (a.flags[par] & 1) {
    const int l = level_of(par, s_off, kMaxLevels) + 1;
    const int pc = a.coord[par];
    const IzSlot z = block_cube(coord_x(pc), coord_y(pc), coord_z(pc), l, par, tid, a.nbr27,
                                a.flags, a.child8);
    if (z.coarse < 0) {
      src = z.real;
    } else if (nvirt > 0) {
      const uint32_t id = cube_id(l, z.key);
      uint32_t h = cube_hash(id, a.bits);
      for (uint32_t probe = 0; probe <= a.mask; ++probe) {
        const uint64_t k = a.hslot[h];
        if (uint32_t(k >> 32) != a.gen) break;
        if (uint32_t(k) == id) {
          src = ncells + a.hval[h];
          break;
        }
        h = (h + 1) & a.mask;
      }
    }
  }
  table[size_t(blockIdx.x) * 216 + tid] = src;
}

static VirtArgs virt_args(Plan& p) {
  VirtArgs a;
  a.depth = p.depth;
  a.lev = p.dlev.as<int>();
  a.cap_cells = p.cap_cells;
  a.coord = p.ccoord.as<int>();
  a.parent = p.cparent.as<int>();
  a.flags = p.cflags.as<int>();
  a.child8 = p.child8.as<int>();
  a.nbr27 = p.nbr27.as<int>();
  a.pb = p.cpb.as<int>();
  a.pe = p.cpe.as<int>();
  a.keys = p.keys.as<uint32_t>();
  a.hslot = p.vhash_keys.as<uint64_t>();
  a.hval = p.vhash_vals.as<int>();
  a.bits = p.vhash_bits;
  a.mask = uint32_t((size_t(1) << p.vhash_bits) - 1);
  a.gen = p.tree_gen;
  a.count = p.vcount.as<int>();
  a.vcubes = p.vcubes.as<int>();
  a.box = p.dbox;
  return a;
}

// the virtual-cube set for the cell arrays' capacity (4 slots per cell, at least 2^13), cleared
// when it is (re)allocated
static void reserve_virt_set(Plan& p, int min_bits, hipStream_t s) {
  int bits = std::max(13, min_bits);
  while ((int64_t(1) << bits) < 4 * p.cap_cells && bits < 30) ++bits;
  if (bits <= p.vhash_bits && p.vhash_keys.p) return;
  p.vhash_bits = bits;
  const size_t slots = size_t(1) << bits;
  p.vhash_keys.release();
  p.vhash_keys.reserve(slots * 8);
  HPM_HIP(hipMemsetAsync(p.vhash_keys.p, 0, slots * 8, s));
  p.vhash_vals.reserve(slots * 4);
  p.vcubes.reserve(slots * 12);
}

static void enqueue_virt_insert(Plan& p, hipStream_t s) {
  // about one parent per workgroup (the parents are fewer than the cells)
  k_virt_insert<<<std::max(1, std::min<int>(int(p.cap_cells), 16384)), 256, 0, s>>>(virt_args(p));
  HPM_LAUNCH_CHECK();
}

void finish_virtual(Plan& p, hipStream_t s) {
  const int first = p.nlevels > 2 ? p.level_off[1] : 0;
  const int nt = p.nlevels > 2 ? p.level_off[p.nlevels - 1] - first : 0;
  const int nv = int(p.nvirt);
  if (nv > 0) {
    ensure_cells(p, p.ncells + nv, p.ncells, s);
    p.vlevel.reserve(size_t(nv) * 4);
    p.vlist.reserve(size_t(nv) * 4);
  }
  p.blocks_first = first;
  if (nt <= 0) return;
  p.blocks.reserve(size_t(nt) * 216 * 4);
  k_virt_finish<<<nt + nblk(nv, 256), 256, 0, s>>>(
      virt_args(p), first, nt, int(p.ncells), nv, p.blocks.as<int>(), p.ccoord.as<int>(),
      p.cpb.as<int>(), p.cpe.as<int>(), p.vlevel.as<int>(), p.vlist.as<int>());
  HPM_LAUNCH_CHECK();
}

}  // namespace hpm
