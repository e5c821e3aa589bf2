// Oct-tree construction on the device (Sec. 1): Morton keys, a stable LSD radix sort of
// (key, input index), levels of real cells by the split rule, child tables, the 27-cube
// neighbourhood of every cell, and the leaf list.
//
// Cells live in one id space with the levels contiguous and each level in Morton order. A cell
// is built from its parent's particle range by binary search for the 8 child key prefixes, so a
// level costs O(cells log n), not O(n). Neighbour entry encoding (27 per cell, x fastest):
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
// Exclusive prefix sum of int32 (block tiles of 2048, recursive over block totals)
// ---------------------------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ int block_exclusive_scan(int v, int* s_wave, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  int wave_pre = 0, all = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    if (w < wave) wave_pre += s_wave[w];
    all += s_wave[w];
  }
  __syncthreads();
  *total = all;
  return wave_pre + x - v;
}

// n is the length, or its upper bound when dn (the length in device memory) is given.
__device__ __forceinline__ int scan_len(int n, const int* dn) { return dn ? min(*dn, n) : n; }

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int* in, int n, const int* dn,
                                                              int* sums) {
  __shared__ int s_wave[kScanThreads / 64];
  n = scan_len(n, dn);
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) v += in[base + k];
  int total;
  (void)block_exclusive_scan(v, s_wave, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tile(const int* in, int* out, int n,
                                                            const int* dn, const int* block_off,
                                                            int* total_out) {
  __shared__ int s_wave[kScanThreads / 64];
  n = scan_len(n, dn);
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    sum += v[k];
  }
  int total;
  int run = block_exclusive_scan(sum, s_wave, &total);
  if (block_off) run += block_off[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (total_out && threadIdx.x == 0) *total_out = (block_off ? block_off[blockIdx.x] : 0) + total;
}

// One workgroup scans up to kScanSingleMax values in chunks of 1024 x 8 with a running offset
// (one launch instead of three for the medium sizes of the tree build; larger inputs scan faster
// on many workgroups).
constexpr int kScanSingleThreads = 1024;
constexpr int kScanSingleMax = kScanSingleThreads * kScanItems;

// the body of k_scan_single (one workgroup of kScanSingleThreads threads)
__device__ __forceinline__ void scan_single(const int* in, int* out, int n, const int* dn,
                                            int* total_out) {
  __shared__ int s_wave[kScanSingleThreads / 64];
  __shared__ int s_run;
  n = scan_len(n, dn);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_run = 0;
  __syncthreads();
  for (int c0 = 0; c0 < n; c0 += kScanSingleThreads * kScanItems) {
    const int base = c0 + threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = (base + k < n) ? in[base + k] : 0;
      sum += v[k];
    }
    int x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    int pre = s_run, all = 0;
    for (int w = 0; w < kScanSingleThreads / 64; ++w) {
      if (w < wave) pre += s_wave[w];
      all += s_wave[w];
    }
    int run = pre + x - sum;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (base + k < n) out[base + k] = run;
      run += v[k];
    }
    __syncthreads();  // every thread has read s_run and s_wave
    if (threadIdx.x == 0) s_run += all;
    __syncthreads();
  }
  if (total_out && threadIdx.x == 0) *total_out = s_run;
}

__global__ __launch_bounds__(kScanSingleThreads) void k_scan_single(const int* in, int* out, int n,
                                                                    const int* dn, int* total_out) {
  scan_single(in, out, n, dn, total_out);
}

static size_t scan_tmp_ints(int n) {
  size_t t = 0;
  while (n > kScanTile) {
    n = (n + kScanTile - 1) / kScanTile;
    t += 2 * size_t(n);
  }
  return t + 16;
}

// Tiles are laid out for n; with dn the kernels scan only the first *dn (<= n) values, and the
// tile sums past them are zero, so the recursion over the sums needs no device length.
static void scan_rec(const int* in, int* out, int n, const int* dn, int* total, int* tmp,
                     hipStream_t s) {
  const int nb = (n + kScanTile - 1) / kScanTile;
  if (nb <= 1) {
    k_scan_tile<<<1, kScanThreads, 0, s>>>(in, out, n, dn, nullptr, total);
    HPM_LAUNCH_CHECK();
    return;
  }
  if (n <= kScanSingleMax) {
    k_scan_single<<<1, kScanSingleThreads, 0, s>>>(in, out, n, dn, total);
    HPM_LAUNCH_CHECK();
    return;
  }
  int* sums = tmp;
  int* sums_scan = tmp + nb;
  k_scan_reduce<<<nb, kScanThreads, 0, s>>>(in, n, dn, sums);
  HPM_LAUNCH_CHECK();
  scan_rec(sums, sums_scan, nb, nullptr, total, tmp + 2 * nb, s);
  k_scan_tile<<<nb, kScanThreads, 0, s>>>(in, out, n, dn, sums_scan, nullptr);
  HPM_LAUNCH_CHECK();
}

// out[i] = sum_{j<i} in[j]; *total (device int, may be null) = sum of all.
void exclusive_scan_i32(const int* in, int* out, int n, int* total, DevBuf& tmp, hipStream_t s) {
  if (n <= 0) return;
  tmp.reserve(scan_tmp_ints(n) * sizeof(int));
  int* t = tmp.as<int>();
  // the last two ints of tmp hold a total when the caller passes none
  scan_rec(in, out, n, nullptr, total, t, s);
}

// ---------------------------------------------------------------------------------------------
// Morton keys
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_keys(int n, const T* x, const T* y, const T* z, double lo0, double lo1,
                       double lo2, double hi0, double hi1, double hi2, double scale, int depth,
                       uint32_t* keys, int* vals, int* box) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double px = double(x[i]), py = double(y[i]), pz = double(z[i]);
  const int maxc = (1 << depth) - 1;
  int bad = 0;
  if (!(isfinite(px) && isfinite(py) && isfinite(pz))) bad = 2;
  else if (!(px >= lo0 && px <= hi0 && py >= lo1 && py <= hi1 && pz >= lo2 && pz <= hi2)) bad = 1;
  if (bad) {
    box[bad == 2 ? Plan::kBoxNonfinite : Plan::kBoxOutOfBox] = 1;
    keys[i] = 0;
    vals[i] = i;
    return;
  }
  // cube index floor((p - lo) * 2^D / size), clamped: the upper face belongs to the last cube
  const int ix = min(max(int(floor((px - lo0) * scale)), 0), maxc);
  const int iy = min(max(int(floor((py - lo1) * scale)), 0), maxc);
  const int iz = min(max(int(floor((pz - lo2) * scale)), 0), maxc);
  keys[i] = morton3(uint32_t(ix), uint32_t(iy), uint32_t(iz), depth);
  vals[i] = i;
}

// ---------------------------------------------------------------------------------------------
// Stable LSD radix sort of (uint32 key, int32 value), 8 bits per pass
// ---------------------------------------------------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsItems = 4;
constexpr int kRsTile = kRsThreads * kRsItems;

__global__ __launch_bounds__(kRsThreads) void k_radix_hist(const uint32_t* keys, int n, int shift,
                                                           int* hist, int nblocks) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kRsTile;
  for (int r = 0; r < kRsItems; ++r) {
    const int i = base + r * kRsThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Items of a tile are taken in rounds of 256 in index order; within a round the rank of an
// item among equal digits comes from wave ballots (lanes) and a per-digit prefix over the four
// waves, so the output order is stable.
__global__ __launch_bounds__(kRsThreads) void k_radix_scatter(const uint32_t* kin, const int* vin,
                                                              uint32_t* kout, int* vout, int n,
                                                              int shift, const int* offs,
                                                              int nblocks) {
  __shared__ int run[256];
  __shared__ int wcnt[kRsThreads / 64][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  run[tid] = offs[tid * nblocks + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  const int base = blockIdx.x * kRsTile;
  for (int r = 0; r < kRsItems; ++r) {
    const int i = base + r * kRsThreads + tid;
    const bool valid = i < n;
    uint32_t key = 0;
    int val = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
    }
    const uint32_t d = (key >> shift) & 255u;
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
      if (pos >= 0 && pos < n) {  // always true for a consistent histogram
        kout[pos] = key;
        vout[pos] = val;
      }
    }
    __syncthreads();
  }
}

// Sorts n (key, value) pairs held in (ka, va); (kb, vb) is scratch of the same size. The result
// ends in (ka, va).
static void radix_sort(uint32_t* ka, int* va, uint32_t* kb, int* vb, int n, int nbits,
                       DevBuf& hist_buf, DevBuf& scan_tmp, hipStream_t s) {
  if (n <= 0) return;
  const int nblocks = (n + kRsTile - 1) / kRsTile;
  hist_buf.reserve(size_t(256) * nblocks * sizeof(int) * 2);
  int* hist = hist_buf.as<int>();
  int* offs = hist + 256 * nblocks;
  const int passes = (nbits + 7) / 8;
  uint32_t* k0 = ka;
  int* v0 = va;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = 8 * pass;
    k_radix_hist<<<nblocks, kRsThreads, 0, s>>>(ka, n, shift, hist, nblocks);
    HPM_LAUNCH_CHECK();
    exclusive_scan_i32(hist, offs, 256 * nblocks, nullptr, scan_tmp, s);
    k_radix_scatter<<<nblocks, kRsThreads, 0, s>>>(ka, va, kb, vb, n, shift, offs, nblocks);
    HPM_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != k0) {
    HPM_HIP(hipMemcpyAsync(k0, ka, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
    HPM_HIP(hipMemcpyAsync(v0, va, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
  }
}

// particle keys: sorted from (tmp_keys, tmp_vals) into (keys, perm); the sorted buffers are
// swapped in rather than copied
static void radix_sort_pairs(Plan& p, int nbits, hipStream_t s) {
  const int n = int(p.n);
  radix_sort(p.tmp_keys.as<uint32_t>(), p.tmp_vals.as<int>(), p.keys.as<uint32_t>(),
             p.perm.as<int>(), n, nbits, p.hist, p.scan_tmp, s);
  p.keys.swap(p.tmp_keys);
  p.perm.swap(p.tmp_vals);
}

template <typename T>
__global__ void k_gather3(int n, const int* perm, const T* x, const T* y, const T* z, T* xs, T* ys,
                          T* zs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = perm[i];
  if (j < 0 || j >= n) return;
  xs[i] = x[j];
  ys[i] = y[j];
  zs[i] = z[j];
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
// particle i - 1. Three launches build every level at once:
//   count: per workgroup of particles, the cells and leaves that start in it on each level; the
//          last workgroup to finish turns them into id bases (levels contiguous, each level in
//          key order, which is Morton order) and writes the level table;
//   emit:  the cells (key, coordinates, particle range, split flag), the leaf list, and a hash of
//          cube id -> cell id;
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
constexpr int kTreeMaxGroups = 2048;      // the count kernel's workgroups (rounds absorb the rest)

struct TreeArgs {
  const uint32_t* keys;  // sorted keys at depth D
  int n;
  int depth;
  int cap;
  int uniform;
  int rounds;           // particles per thread: workgroup b takes [b rounds 256, (b+1) rounds 256)
  int* blk;             // [workgroups][kTreeSeq]: counts, then id bases
  int* done;            // workgroups of the count kernel finished (its last one resets it)
  int* lev;             // level table
  int* box;             // mailbox words
  int* zero_words;      // cleared by the count kernel for the later steps of the build (4 ints)
  unsigned long long* zero_pairs;  // near-zone pair count, likewise
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

// first j in (i, hi] with keys[j] >= v (hi if none below hi); keys[i] < v
__device__ __forceinline__ int gallop_fwd(const uint32_t* keys, int i, int hi, uint32_t v) {
  int lo = i + 1, step = 1, j = i + 1;
  while (j < hi && keys[j] < v) {
    lo = j + 1;
    step <<= 1;
    j = i + step;
  }
  return lower_bound_u32(keys, lo, min(j, hi), v);
}

// first j in [0, i] with keys[j] >= v; keys[i] >= v
__device__ __forceinline__ int gallop_back(const uint32_t* keys, int i, uint32_t v) {
  int hi = i, step = 1, j = i - 1;
  while (j >= 0 && keys[j] >= v) {
    hi = j;
    step <<= 1;
    j = i - step;
  }
  return lower_bound_u32(keys, max(j + 1, 0), hi, v);
}

// The runs that start at one particle, walked level by level.
struct Walk {
  uint32_t key;
  int i;
  int lo;    // first level at which a cell starts here
  int end;   // end of the run of the previous level
  bool live; // cells start here at the levels still to come (until the leaf)
};

__device__ __forceinline__ Walk walk_init(const TreeArgs& a, int i) {
  Walk w{0u, i, kMaxLevels, 0, false};
  if (i >= a.n) return w;
  const uint32_t k = a.keys[i];
  w.key = k;
  int d = 0;
  if (i > 0) {
    const uint32_t x = k ^ a.keys[i - 1];
    if (x == 0u) return w;  // same cube as the previous particle at every level
    d = a.depth - (31 - __clz(int(x))) / 3;
  }
  int end = a.n;
  if (d >= 1 && !a.uniform) {
    // the parent run (level d - 1) must be split: more than cap particles
    const int sh = 3 * (a.depth - d + 1);
    const uint32_t pre = k >> sh;
    const int e = gallop_fwd(a.keys, i, a.n, (pre + 1u) << sh);
    const int b = gallop_back(a.keys, i, pre << sh);
    if (e - b <= a.cap) return w;
    end = e;
  }
  w.lo = d;
  w.end = end;
  w.live = true;
  return w;
}

// level l of the walk (called for l = 0, 1, ... in order): a cell starts here (cell), it is a
// leaf (leaf), with cnt particles
__device__ __forceinline__ void walk_step(const TreeArgs& a, Walk& w, int l, bool& cell, bool& leaf,
                                          int& cnt) {
  cell = leaf = false;
  cnt = 0;
  if (!w.live || l < w.lo) return;
  const int sh = 3 * (a.depth - l);
  const int e = (l == 0) ? a.n : gallop_fwd(a.keys, w.i, w.end, ((w.key >> sh) + 1u) << sh);
  cnt = e - w.i;
  cell = true;
  leaf = a.uniform ? (l >= a.depth) : (cnt <= a.cap || l >= a.depth);
  w.end = e;
  if (leaf) w.live = false;
}

// exclusive scan of one value per thread over the workgroup (kTreeThreads), and the total
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
  for (int w = 0; w < kTreeThreads / 64; ++w) {
    if (w < wave) pre += s_w[w];
    all += s_w[w];
  }
  __syncthreads();
  total = all;
  return pre + x - v;
}

__global__ __launch_bounds__(kTreeThreads) void k_tree_count(TreeArgs a) {
  __shared__ int s_cnt[kTreeSeq];
  __shared__ int s_w[kTreeThreads / 64];
  __shared__ int s_last;
  __shared__ int s_tot[kTreeSeq];
  __shared__ int s_off[kTreeSeq];
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < kTreeSeq) s_cnt[tid] = 0;
  __syncthreads();
  for (int r = 0; r < a.rounds; ++r) {
    const int i = (blockIdx.x * a.rounds + r) * kTreeThreads + tid;
    Walk w = walk_init(a, i);
    for (int l = 0; l < kMaxLevels; ++l) {
      bool cell, leaf;
      int cnt;
      walk_step(a, w, l, cell, leaf, cnt);
      const uint64_t mc = __ballot(cell), ml = __ballot(leaf);
      if (lane == 0 && mc) atomicAdd(&s_cnt[l], __popcll(mc));
      if (lane == 0 && ml) atomicAdd(&s_cnt[kMaxLevels + l], __popcll(ml));
    }
  }
  __syncthreads();
  if (tid < kTreeSeq) a.blk[size_t(blockIdx.x) * kTreeSeq + tid] = s_cnt[tid];
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = (atomicAdd(a.done, 1) == int(gridDim.x) - 1);
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // the last workgroup: bases of every workgroup, level-major (thread t takes a chunk of them)
  const int nb = gridDim.x, per = (nb + kTreeThreads - 1) / kTreeThreads;
  const int b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
  for (int q = 0; q < kTreeSeq; ++q) {
    int sum = 0;
    for (int b = b0; b < b1; ++b) sum += a.blk[size_t(b) * kTreeSeq + q];
    int tot;
    int run = group_scan(sum, s_w, tot);
    if (tid == 0) s_tot[q] = tot;
    for (int b = b0; b < b1; ++b) {
      const int c = a.blk[size_t(b) * kTreeSeq + q];
      a.blk[size_t(b) * kTreeSeq + q] = run;  // within the level; the level offset is added below
      run += c;
    }
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
    int* lev = a.lev;
    for (int l = 0; l < 16; ++l) {
      lev[kLevOff + l] = l < kMaxLevels ? s_off[l] : oc;
      lev[kLevCnt + l] = l < kMaxLevels ? s_tot[l] : 0;
    }
    lev[kLevCells] = oc;
    lev[kLevLeaves] = ol;
    lev[kLevLeavesLt2] = s_tot[kMaxLevels] + s_tot[kMaxLevels + 1];
    int nlev = 0, ps = 0;
    for (int l = 0; l < 12; ++l) {
      lev[kLevLeafOff + l] = l < kMaxLevels ? s_off[kMaxLevels + l] : ol;
      lev[kLevSplitOff + l] = ps;  // split cells of levels 1 .. l-1
      if (l >= 1 && l < kMaxLevels) ps += s_tot[l] - s_tot[kMaxLevels + l];
      if (l < kMaxLevels && s_tot[l] > 0) nlev = l + 1;
    }
    for (int w = 0; w < kLevWords; ++w) a.box[Plan::kBoxLev + w] = lev[w];
    a.box[Plan::kBoxLeaves] = ol;
    a.box[Plan::kBoxLeavesLt2] = lev[kLevLeavesLt2];
    for (int l = 1; l < nlev; ++l) a.box[Plan::kBoxCellLevels + l] = lev[kLevSplitOff + l];
    for (int w = 0; w < 4; ++w) a.zero_words[w] = 0;
    *a.zero_pairs = 0ull;
    *a.done = 0;
  }
  __syncthreads();
  for (int b = b0; b < b1; ++b)
    for (int q = 0; q < kTreeSeq; ++q) a.blk[size_t(b) * kTreeSeq + q] += s_off[q];
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
  if (int64_t(a.lev[kLevCells]) > a.cap_cells) return;  // the host grows the arrays and re-runs
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < kTreeSeq) s_run[tid] = a.blk[size_t(blockIdx.x) * kTreeSeq + tid];
  if (tid < kLevWords) s_lev[tid] = a.lev[tid];
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  __syncthreads();
  for (int r = 0; r < a.rounds; ++r) {
    const int i = (blockIdx.x * a.rounds + r) * kTreeThreads + tid;
    Walk w = walk_init(a, i);
    for (int l = 0; l < kMaxLevels; ++l) {
      bool cell, leaf;
      int cnt;
      walk_step(a, w, l, cell, leaf, cnt);
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
        chash_insert(a, cube_id(l, key), id);
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

  const double scale = double(1 << D) / pr.box_size;
  const double hi0 = pr.box_lo[0] + pr.box_size, hi1 = pr.box_lo[1] + pr.box_size,
               hi2 = pr.box_lo[2] + pr.box_size;
  if (p.prec == HPM_F32) {
    k_keys<float><<<nblk(n, 256), 256, 0, s>>>(n, (const float*)x, (const float*)y,
                                               (const float*)z, pr.box_lo[0], pr.box_lo[1],
                                               pr.box_lo[2], hi0, hi1, hi2, scale, D,
                                               p.tmp_keys.as<uint32_t>(), p.tmp_vals.as<int>(),
                                               p.dbox);
  } else {
    k_keys<double><<<nblk(n, 256), 256, 0, s>>>(n, (const double*)x, (const double*)y,
                                                (const double*)z, pr.box_lo[0], pr.box_lo[1],
                                                pr.box_lo[2], hi0, hi1, hi2, scale, D,
                                                p.tmp_keys.as<uint32_t>(), p.tmp_vals.as<int>(),
                                                p.dbox);
  }
  HPM_LAUNCH_CHECK();
  // invalid positions got key 0, so the build below stays well defined; the flags are checked
  // at the synchronisation after the levels

  radix_sort_pairs(p, 3 * D, s);

  p.xs.reserve(size_t(n) * p.elem);
  p.ys.reserve(size_t(n) * p.elem);
  p.zs.reserve(size_t(n) * p.elem);
  p.ms.reserve(size_t(n) * p.elem);
  if (p.prec == HPM_F32)
    k_gather3<float><<<nblk(n, 256), 256, 0, s>>>(n, p.perm.as<int>(), (const float*)x,
                                                  (const float*)y, (const float*)z,
                                                  p.xs.as<float>(), p.ys.as<float>(),
                                                  p.zs.as<float>());
  else
    k_gather3<double><<<nblk(n, 256), 256, 0, s>>>(n, p.perm.as<int>(), (const double*)x,
                                                   (const double*)y, (const double*)z,
                                                   p.xs.as<double>(), p.ys.as<double>(),
                                                   p.zs.as<double>());
  HPM_LAUNCH_CHECK();

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
  reserve_cleared(p.tree_done, 16, s);
  p.dlev.reserve(kLevWords * sizeof(int));
  a.blk = p.tree_blk.as<int>();
  a.done = p.tree_done.as<int>();
  a.lev = p.dlev.as<int>();
  a.box = p.dbox;
  p.vcount.reserve(4 * sizeof(int));  // cleared by the count kernel
  p.pairs.reserve(16);
  a.zero_words = p.vcount.as<int>();
  a.zero_pairs = p.pairs.as<unsigned long long>();
  k_tree_count<<<groups, kTreeThreads, 0, s>>>(a);
  HPM_LAUNCH_CHECK();
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
    HPM_HIP(hipMemsetAsync(p.vcount.p, 0, 3 * sizeof(int), s));
    enqueue_virt_insert(p, s);
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
  p.dlevel.reserve(sizeof(p.level_off));
  HPM_HIP(hipMemcpyAsync(p.dlevel.p, p.level_off, sizeof(p.level_off), hipMemcpyHostToDevice, s));
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
  int* count;            // [0] cubes listed, [1] the set is full, [2] finish counter
  uint32_t* vkeys;       // cube id of each v
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
// and records the id at vkeys[v]. A full set raises count[1]. The last workgroup to finish copies
// the two words to the mailbox.
__global__ __launch_bounds__(256) void k_virt_insert(VirtArgs a) {
  __shared__ int s_off[kMaxLevels + 1];
  __shared__ int s_last;
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
    const int vb = lower_bound_u32(a.keys, cb, ce, z.key << shift);
    const int ve = lower_bound_u32(a.keys, vb, ce, (z.key + 1u) << shift);
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
        a.vkeys[v] = id;
        placed = true;
        break;
      }
      // the slot changed under us (another insertion of this build): look at it again
    }
    if (!placed) atomicExch(&a.count[1], 1);
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = (atomicAdd(&a.count[2], 1) == int(gridDim.x) - 1);
  __syncthreads();
  if (!s_last || tid != 0) return;
  __threadfence();
  a.box[Plan::kBoxVirt] = __hip_atomic_load(&a.count[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  a.box[Plan::kBoxVirtFull] = __hip_atomic_load(&a.count[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  a.count[2] = 0;
}

// Workgroups [0, nt): the source gridlet id of every slot of the 6^3 block of each parent of
// targets: a real cell id, ncells + v for virtual cube v (found in the hash set), or -1 (empty
// position, outside the box, or not a parent). Workgroups from nt on: coordinates, particle range
// and level of virtual cube v, stored at cell id ncells + v.
__global__ __launch_bounds__(256) void k_virt_finish(VirtArgs a, int first, int nt, int ncells,
                                                     int nvirt, int* table, int* coord, int* pb,
                                                     int* pe, int* vlevel, int* vlist, int n) {
  __shared__ int s_off[kMaxLevels + 1];
  const int tid = threadIdx.x;
  if (int(blockIdx.x) >= nt) {
    const int v = (blockIdx.x - nt) * 256 + tid;
    if (v >= nvirt) return;
    const uint32_t id = a.vkeys[v];
    const int l = cube_id_level(id);
    const uint32_t key = id ^ (1u << (3 * l));
    int x = 0, y = 0, z = 0;
    for (int b = 0; b < l; ++b) {
      x |= int((key >> (3 * b)) & 1u) << b;
      y |= int((key >> (3 * b + 1)) & 1u) << b;
      z |= int((key >> (3 * b + 2)) & 1u) << b;
    }
    const int shift = 3 * (a.depth - l);
    const int b0 = lower_bound_u32(a.keys, 0, n, key << shift);
    const int e0 = lower_bound_u32(a.keys, b0, n, (key + 1u) << shift);
    coord[ncells + v] = pack_coord(x, y, z);
    pb[ncells + v] = b0;
    pe[ncells + v] = e0;
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
  a.vkeys = p.vkeys.as<uint32_t>();
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
  p.vkeys.reserve(slots * 4);
}

static void enqueue_virt_insert(Plan& p, hipStream_t s) {
  k_virt_insert<<<std::max(1, std::min<int>(int(p.cap_cells), 2048)), 256, 0, s>>>(virt_args(p));
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
      p.cpb.as<int>(), p.cpe.as<int>(), p.vlevel.as<int>(), p.vlist.as<int>(), int(p.n));
  HPM_LAUNCH_CHECK();
}

}  // namespace hpm
