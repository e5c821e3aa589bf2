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

// The same over the first *dn values (device memory, at most nmax); tmp must already hold the
// scratch for nmax (no allocation here, so that it can run between kernels still in flight).
// Up to kScanDnSingleMax the scan is one workgroup that stops at *dn: a level's cell count is
// usually far below the host's bound, and one launch replaces the three of the tiled scan.
constexpr int kScanDnSingleMax = 8 * kScanSingleMax;

static void exclusive_scan_i32_dn(const int* in, int* out, int nmax, const int* dn, int* total,
                                  DevBuf& tmp, hipStream_t s) {
  if (nmax <= 0) return;
  if (nmax <= kScanDnSingleMax) {
    k_scan_single<<<1, kScanSingleThreads, 0, s>>>(in, out, nmax, dn, total);
    HPM_LAUNCH_CHECK();
    return;
  }
  if (tmp.bytes < scan_tmp_ints(nmax) * sizeof(int)) fail(HPM_ERR_DEVICE, "scan scratch too small");
  scan_rec(in, out, nmax, dn, total, tmp.as<int>(), s);
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

// Level table in device memory, written by the level kernels as the tree grows, so that the
// level loop runs without host round trips: first cell id and cell count of each level, and the
// level whose children did not fit the cell arrays (-1: none; every later level kernel then
// returns, and the host grows the arrays and resumes there).
constexpr int kLevOff = 0, kLevCnt = 16, kLevOverflow = 32, kLevWords = 40;

__global__ void k_root(int n, CellArrays c, int* lev) {
  const int t = threadIdx.x;
  if (t < 27) c.nbr27[t] = (t == 13) ? 0 : -1;
  if (t < kLevWords) lev[t] = (t == kLevCnt) ? 1 : (t == kLevOverflow ? -1 : 0);
  if (t == 0) {
    c.key[0] = 0;
    c.coord[0] = 0;
    c.pb[0] = 0;
    c.pe[0] = n;
    c.parent[0] = -1;
  }
}

__global__ void k_lev_resume(int* lev) { lev[kLevOverflow] = -1; }

__device__ void level_nbr(int l, int off, int cnt, CellArrays c);

// Split decision and the 9 boundaries of the child ranges of each cell of level l: eight lanes
// per cell, lane k finds the first particle of child octant k by binary search in the cell's
// (key-sorted) range. Grid-stride over the level's cells (count from the level table). For
// l >= 1 the same launch first fills the level's 27-cube neighbourhoods (they read only level
// l-1, which the previous launches completed).
__device__ __forceinline__ void level_split(int l, int depth, int uniform, int cap, const int* lev,
                                            const uint32_t* keys, CellArrays c, int* bounds,
                                            int* nchild) {
  const int off = lev[kLevOff + l], cnt = lev[kLevCnt + l];
  if (l >= 1) level_nbr(l, off, cnt, c);
  for (int64_t t0 = int64_t(blockIdx.x) * blockDim.x; t0 < int64_t(cnt) * 8;
       t0 += int64_t(gridDim.x) * blockDim.x) {
    const int64_t t = t0 + threadIdx.x;
    const int i = int(t >> 3), k = int(t & 7);
    const bool live = i < cnt;
    int b = 0, nonempty = 0;
    bool split = false;
    int pe = 0;
    if (live) {
      const int g = off + i;
      const int pb = c.pb[g];
      pe = c.pe[g];
      split = uniform ? (l < depth) : ((pe - pb) > cap && l < depth);
      if (k == 0) c.flags[g] = split ? 1 : 0;
      if (split) {
        const int shift = 3 * (depth - l - 1);
        const uint32_t base = c.key[g] << 3;
        b = (k == 0) ? pb : lower_bound_u32(keys, pb, pe, (base + uint32_t(k)) << shift);
        bounds[i * 9 + k] = b;
        if (k == 7) bounds[i * 9 + 8] = pe;
      }
    }
    // child k is nonempty if the next boundary is past this one (lanes k+1 of the same cell)
    const int next = __shfl_down(b, 1, 8);
    if (live && split) nonempty = ((k == 7) ? pe : next) > b ? 1 : 0;
    int nc = nonempty;
    nc += __shfl_xor(nc, 1, 8);
    nc += __shfl_xor(nc, 2, 8);
    nc += __shfl_xor(nc, 4, 8);
    if (live && k == 0) nchild[i] = split ? nc : 0;
  }
}

__global__ void k_level_split(int l, int depth, int uniform, int cap, const int* lev,
                              const uint32_t* keys, CellArrays c, int* bounds, int* nchild) {
  if (lev[kLevOverflow] >= 0) return;
  level_split(l, depth, uniform, cap, lev, keys, c, bounds, nchild);
}

// Children of the cells of level l at ids off_next + childoff[i] + r (the scan of the split
// counts left the number of level-(l+1) cells in the table); flags the overflow instead when they
// do not fit in cap cells.
__device__ __forceinline__ void level_emit(int l, int cap_cells, int* lev, const int* bounds,
                                           const int* childoff, CellArrays c) {
  const int off = lev[kLevOff + l], cnt = lev[kLevCnt + l], total = lev[kLevCnt + l + 1];
  const int off_next = off + cnt;
  if (int64_t(off_next) + total > cap_cells) {
    if (blockIdx.x == 0 && threadIdx.x == 0) lev[kLevOverflow] = l;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) lev[kLevOff + l + 1] = off_next;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
    const int g = off + i;
    const bool split = c.flags[g] & 1;
    const int cx = coord_x(c.coord[g]), cy = coord_y(c.coord[g]), cz = coord_z(c.coord[g]);
    int r = 0;
    for (int k = 0; k < 8; ++k) {
      int id = -1;
      if (split) {
        const int b0 = bounds[i * 9 + k], b1 = bounds[i * 9 + k + 1];
        if (b1 > b0) {
          id = off_next + childoff[i] + r++;
          c.key[id] = (c.key[g] << 3) | uint32_t(k);
          c.coord[id] = pack_coord(2 * cx + (k & 1), 2 * cy + ((k >> 1) & 1), 2 * cz + ((k >> 2) & 1));
          c.pb[id] = b0;
          c.pe[id] = b1;
          c.parent[id] = g;
        }
      }
      c.child8[g * 8 + k] = id;
    }
  }
}

__global__ void k_level_emit(int l, int cap_cells, int* lev, const int* bounds, const int* childoff,
                             CellArrays c) {
  if (lev[kLevOverflow] >= 0) return;
  level_emit(l, cap_cells, lev, bounds, childoff, c);
}


// 27-cube neighbourhood of the cells of level l (>= 1) from the parent's neighbourhood: one
// thread per (cell, neighbour) entry, grid-stride.
__device__ void level_nbr(int l, int off, int cnt, CellArrays c) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < int64_t(cnt) * 27;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(t / 27), j = int(t % 27);
    const int dx = j % 3 - 1, dy = (j / 3) % 3 - 1, dz = j / 9 - 1;
    const int g = off + i;
    const int pc = c.coord[g];
    const int x = coord_x(pc), y = coord_y(pc), z = coord_z(pc);
    const int par = c.parent[g];
    const int side = 1 << l;
    const int qx = x + dx, qy = y + dy, qz = z + dz;
    int v = -1;
    if (qx >= 0 && qy >= 0 && qz >= 0 && qx < side && qy < side && qz < side) {
      const int ox = (qx >> 1) - (x >> 1), oy = (qy >> 1) - (y >> 1), oz = (qz >> 1) - (z >> 1);
      const int e = c.nbr27[par * 27 + (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)];
      if (e >= 0) {
        if (c.flags[e] & 1) v = c.child8[e * 8 + ((qx & 1) | ((qy & 1) << 1) | ((qz & 1) << 2))];
        else v = -2 - e;
      } else {
        v = e;
      }
    }
    c.nbr27[g * 27 + j] = v;
  }
}

__global__ void k_leaf_flags(int ncells, const int* flags, int* isleaf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncells) isleaf[i] = (flags[i] & 1) ? 0 : 1;
}

// leaf list; the cell with id first2 (the first of level 2) reports how many leaves precede it
__global__ void k_leaf_compact(int ncells, const int* flags, const int* pos, int* leaves,
                               int first2, int* lt2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncells && i == first2) *lt2 = pos[i];
  if (i < ncells && !(flags[i] & 1)) leaves[pos[i]] = i;
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

static inline int nblk(int64_t n, int t) { return int((n + t - 1) / t); }

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
  // at the first synchronisation of the level loop

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

  // levels, all enqueued back to back: every level kernel reads its level's cell range from the
  // device table, and the host waits once, at the end (or where the cells outgrew the arrays)
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
  p.dlev.reserve(kLevWords * sizeof(int));
  int* lev = p.dlev.as<int>();
  auto level_scratch = [&](int64_t keep) {
    const size_t c = size_t(p.cap_cells);
    p.bounds.grow(c * 9 * 4, size_t(keep) * 9 * 4, s);
    p.childoff.grow(c * 4, size_t(keep) * 4, s);
    p.nchild.grow(c * 4, 0, s);
    p.scan_tmp.reserve(scan_tmp_ints(int(std::min<int64_t>(c, n))) * sizeof(int));
  };
  level_scratch(0);
  k_root<<<1, 64, 0, s>>>(n, cells_of(p), lev);
  HPM_LAUNCH_CHECK();
  auto grid = [](int64_t work, int t) {
    return int(std::max<int64_t>(1, std::min<int64_t>((work + t - 1) / t, 4096)));
  };
  // levels from..to; the kernels of a level with no cells return at once, but each launch still
  // costs, so adaptive trees are enqueued to a depth their size suggests first, and the rest
  // only if the table read back says the tree goes deeper
  auto enqueue = [&](int from, bool resume_emit, int to) {
    const CellArrays c = cells_of(p);
    for (int l = from; l <= to; ++l) {
      // cells of level l: at most 8^l, n (nonempty) and the capacity
      const int64_t ub = std::min<int64_t>({int64_t(1) << (3 * l), int64_t(n), p.cap_cells});
      if (!(l == from && resume_emit)) {
        k_level_split<<<grid(ub * 27, 256), 256, 0, s>>>(l, D, uniform ? 1 : 0, pr.leaf_capacity,
                                                       lev, p.keys.as<uint32_t>(), c,
                                                       p.bounds.as<int>(), p.nchild.as<int>());
        HPM_LAUNCH_CHECK();
        exclusive_scan_i32_dn(p.nchild.as<int>(), p.childoff.as<int>(), int(ub),
                              lev + kLevCnt + l, lev + kLevCnt + l + 1, p.scan_tmp, s);
      }
      k_level_emit<<<grid(ub, 128), 128, 0, s>>>(l, int(p.cap_cells), lev, p.bounds.as<int>(),
                                                 p.childoff.as<int>(), c);
      HPM_LAUNCH_CHECK();
    }
  };
  const int* hl = p.hbox + Plan::kBoxLev;
  int to = D;
  if (!uniform) {
    // log8(n / capacity) levels hold the leaves of an even density; Plummer-like concentration
    // adds a few (2^18 Plummer particles, 64 per leaf: 8 levels past the root)
    int est = 0;
    for (int64_t cells = 1; cells * std::max(1, pr.leaf_capacity) < int64_t(n); cells *= 8) ++est;
    to = std::min(D, est + 5);
  }
  enqueue(0, false, to);
  for (bool first = true;; first = false) {
    HPM_HIP(hipMemcpyAsync(p.hbox + Plan::kBoxLev, lev, kLevWords * sizeof(int),
                           hipMemcpyDeviceToHost, s));
    sync_box(p, s);
    if (first) {
      if (p.hbox[Plan::kBoxNonfinite]) fail(HPM_ERR_NONFINITE, "a particle position is not finite");
      if (p.hbox[Plan::kBoxOutOfBox])
        fail(HPM_ERR_OUT_OF_BOX, "a particle position is outside the box");
    }
    const int ov = hl[kLevOverflow];
    if (ov < 0) {
      if (to < D && hl[kLevCnt + to + 1] > 0) {  // the tree goes deeper than enqueued
        const int from = to + 1;
        to = D;
        enqueue(from, false, to);
        continue;
      }
      break;
    }
    // the children of level ov did not fit: keep the levels up to ov (and ov's split), grow,
    // and emit from level ov on
    const int64_t keep = int64_t(hl[kLevOff + ov]) + hl[kLevCnt + ov];
    const int64_t need = keep + hl[kLevCnt + ov + 1];
    ensure_cells(p, need + need / 2 + 64, keep, s);
    level_scratch(hl[kLevCnt + ov]);
    k_lev_resume<<<1, 1, 0, s>>>(lev);
    HPM_LAUNCH_CHECK();
    enqueue(ov, true, to);
  }
  p.nlevels = 0;
  for (int l = 0; l <= D; ++l) {
    if (hl[kLevCnt + l] <= 0) break;
    p.level_off[l] = hl[kLevOff + l];
    p.nlevels = l + 1;
  }
  p.ncells = int64_t(p.level_off[p.nlevels - 1]) + hl[kLevCnt + p.nlevels - 1];
  for (int l = p.nlevels; l <= kMaxLevelsHost; ++l) p.level_off[l] = int(p.ncells);
  p.dlevel.reserve(sizeof(p.level_off));
  HPM_HIP(hipMemcpyAsync(p.dlevel.p, p.level_off, sizeof(p.level_off), hipMemcpyHostToDevice, s));

  // leaf list (global-id order, so leaves of levels 0 and 1 come first)
  const int nc = int(p.ncells);
  p.nchild.reserve(size_t(nc) * 4);
  p.childoff.reserve(size_t(nc) * 4);
  k_leaf_flags<<<nblk(nc, 256), 256, 0, s>>>(nc, p.cflags.as<int>(), p.nchild.as<int>());
  HPM_LAUNCH_CHECK();
  exclusive_scan_i32(p.nchild.as<int>(), p.childoff.as<int>(), nc, p.dbox + Plan::kBoxLeaves,
                     p.scan_tmp, s);
  p.leaves.reserve(size_t(nc) * 4);  // at most one leaf per cell
  const int first2 = p.nlevels > 2 ? p.level_off[2] : -1;
  k_leaf_compact<<<nblk(nc, 256), 256, 0, s>>>(nc, p.cflags.as<int>(), p.childoff.as<int>(),
                                               p.leaves.as<int>(), first2,
                                               p.dbox + Plan::kBoxLeavesLt2);
  HPM_LAUNCH_CHECK();
  // the counts are read by build_virtual after its first synchronisation
}

static void read_leaf_counts(Plan& p) {
  p.nleaves = p.hbox[Plan::kBoxLeaves];
  p.nleaves_lt2 = (p.nlevels > 2) ? p.hbox[Plan::kBoxLeavesLt2] : p.nleaves;
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
  int first_target;
  int depth;
  int nlevels;
  const int* level_off;
  const int* coord;
  const int* parent;
  const int* flags;
  const int* child8;
  const int* nbr27;
  const int* pb;
  const int* pe;
  const uint32_t* keys;  // sorted particle keys at depth D
  uint32_t* hkeys;       // hash set: cube id per slot (kNoCube: empty)
  int* hvals;            // hash set: v per slot
  uint32_t mask;         // slots - 1
  int bits;              // slots = 2^bits
};

constexpr uint32_t kNoCube = 0xffffffffu;  // cube ids are below 2^31

// multiplicative (Fibonacci) hashing: the top "bits" bits of id times 2^32 / golden ratio
__device__ __forceinline__ uint32_t cube_hash(uint32_t id, int bits) {
  return (id * 0x9E3779B1u) >> (32 - bits);
}

// One workgroup per cell of levels 1 .. L-2 (the possible parents of targets), one thread per
// slot of its 6^3 block: a nonempty virtual cube in the interaction zone of some child (every
// block cube except the 8 children's own positions) joins the set; the thread that adds a new id
// takes the next index v and records the id at vkeys[v]. A full set raises *full.
__global__ __launch_bounds__(256) void k_virt_insert(VirtArgs a, int* count, uint32_t* vkeys,
                                                     int* full) {
  __shared__ int s_off[kMaxLevels + 1];
  const int tid = threadIdx.x;
  if (tid <= kMaxLevels) s_off[tid] = a.level_off[tid];
  __syncthreads();
  const int par = a.first_target + blockIdx.x;
  if (tid >= 216 || !(a.flags[par] & 1)) return;
  const int l = level_of(par, s_off, a.nlevels) + 1;  // level of the block's cubes
  const int bx = tid % 6, by = (tid / 6) % 6, bz = tid / 36;
  if (bx >= 2 && bx <= 3 && by >= 2 && by <= 3 && bz >= 2 && bz <= 3) return;  // children
  const int pc = a.coord[par];
  const IzSlot z = block_cube(coord_x(pc), coord_y(pc), coord_z(pc), l, par, tid, a.nbr27, a.flags,
                              a.child8);
  if (z.coarse < 0) return;
  const int shift = 3 * (a.depth - l);
  const int cb = a.pb[z.coarse], ce = a.pe[z.coarse];
  const int vb = lower_bound_u32(a.keys, cb, ce, z.key << shift);
  const int ve = lower_bound_u32(a.keys, vb, ce, (z.key + 1u) << shift);
  if (ve <= vb) return;
  const uint32_t id = cube_id(l, z.key);
  uint32_t h = cube_hash(id, a.bits);
  for (uint32_t probe = 0; probe <= a.mask; ++probe) {
    const uint32_t prev = atomicCAS(&a.hkeys[h], kNoCube, id);
    if (prev == kNoCube) {
      const int v = atomicAdd(count, 1);
      a.hvals[h] = v;
      vkeys[v] = id;
      return;
    }
    if (prev == id) return;
    h = (h + 1) & a.mask;
  }
  atomicExch(full, 1);
}

__global__ void k_copy_words(const int* src, int* dst, int count) {
  if (int(threadIdx.x) < count) dst[threadIdx.x] = src[threadIdx.x];
}

// coordinates, particle range and level of virtual cube v, stored at cell id ncells + v
__global__ void k_virt_cells(int nv, const uint32_t* vids, int depth, int n, const uint32_t* keys,
                             int ncells, int* coord, int* pb, int* pe, int* vlevel, int* vlist) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const uint32_t id = vids[v];
  const int l = cube_id_level(id);
  const uint32_t key = id ^ (1u << (3 * l));
  int x = 0, y = 0, z = 0;
  for (int b = 0; b < l; ++b) {
    x |= int((key >> (3 * b)) & 1u) << b;
    y |= int((key >> (3 * b + 1)) & 1u) << b;
    z |= int((key >> (3 * b + 2)) & 1u) << b;
  }
  const int shift = 3 * (depth - l);
  const int b0 = lower_bound_u32(keys, 0, n, key << shift);
  const int e0 = lower_bound_u32(keys, b0, n, (key + 1u) << shift);
  coord[ncells + v] = pack_coord(x, y, z);
  pb[ncells + v] = b0;
  pe[ncells + v] = e0;
  vlevel[v] = l;
  vlist[v] = ncells + v;
}

// Source gridlet id of every slot of the 6^3 block of each parent of targets: a real cell id,
// ncells + v for virtual cube v (found in the hash set), or -1 (empty position, outside the box,
// or not a parent).
__global__ __launch_bounds__(256) void k_block_table(VirtArgs a, int ncells, int nvirt, int* table) {
  __shared__ int s_off[kMaxLevels + 1];
  const int tid = threadIdx.x;
  if (tid <= kMaxLevels) s_off[tid] = a.level_off[tid];
  __syncthreads();
  if (tid >= 216) return;
  const int par = a.first_target + blockIdx.x;
  int src = -1;
  if (a.flags[par] & 1) {
    const int l = level_of(par, s_off, a.nlevels) + 1;
    const int pc = a.coord[par];
    const IzSlot z = block_cube(coord_x(pc), coord_y(pc), coord_z(pc), l, par, tid, a.nbr27,
                                a.flags, a.child8);
    if (z.coarse < 0) {
      src = z.real;
    } else if (nvirt > 0) {
      const uint32_t id = cube_id(l, z.key);
      uint32_t h = cube_hash(id, a.bits);
      for (uint32_t probe = 0; probe <= a.mask; ++probe) {
        const uint32_t k = a.hkeys[h];
        if (k == id) {
          src = ncells + a.hvals[h];
          break;
        }
        if (k == kNoCube) break;
        h = (h + 1) & a.mask;
      }
    }
  }
  table[size_t(blockIdx.x) * 216 + tid] = src;
}

static void build_block_table(Plan& p, const VirtArgs& a, int nt, hipStream_t s) {
  p.blocks.reserve(size_t(nt) * 216 * 4);
  p.blocks_first = a.first_target;
  k_block_table<<<nt, 256, 0, s>>>(a, int(p.ncells), int(p.nvirt), p.blocks.as<int>());
  HPM_LAUNCH_CHECK();
}

void build_virtual(Plan& p, hipStream_t s) {
  p.nvirt = 0;
  // parents of targets: cells of levels 1 .. nlevels-2
  const int first = p.nlevels > 2 ? p.level_off[1] : 0;
  const int nt = p.nlevels > 2 ? p.level_off[p.nlevels - 1] - first : 0;
  if (nt <= 0) {
    sync_box(p, s);
    read_leaf_counts(p);
    return;
  }
  VirtArgs a;
  a.first_target = first;
  a.depth = p.depth;
  a.nlevels = p.nlevels;
  a.level_off = p.dlevel.as<int>();
  a.coord = p.ccoord.as<int>();
  a.parent = p.cparent.as<int>();
  a.flags = p.cflags.as<int>();
  a.child8 = p.child8.as<int>();
  a.nbr27 = p.nbr27.as<int>();
  a.pb = p.cpb.as<int>();
  a.pe = p.cpe.as<int>();
  a.keys = p.keys.as<uint32_t>();
  a.hkeys = nullptr;
  a.hvals = nullptr;
  a.mask = 0;
  a.bits = 0;
  if (p.prob.uniform_depth > 0) {
    // a uniform tree splits every occupied cell above its last level: every leaf is on the last
    // level, and no block cube lies inside a coarser leaf, so there are no virtual cubes and the
    // leaf counts follow from the level table (no host round trip)
    p.nleaves = p.level_off[p.nlevels] - p.level_off[p.nlevels - 1];
    p.nleaves_lt2 = 0;  // nlevels > 2 here
    build_block_table(p, a, nt, s);
    return;
  }
  // the set starts at 4 slots per cell (at least 2^13) and grows by 4x when a build fills it
  int bits = 13;
  while ((int64_t(1) << bits) < 4 * p.ncells && bits < 30) ++bits;
  p.vhash_bits = std::max(p.vhash_bits, bits);
  int nv = 0;
  for (;;) {
    const size_t slots = size_t(1) << p.vhash_bits;
    p.vhash_keys.reserve(slots * 4);
    p.vhash_vals.reserve(slots * 4);
    p.vkeys.reserve(slots * 4);
    HPM_HIP(hipMemsetAsync(p.vhash_keys.p, 0xff, slots * 4, s));
    // the count and the full flag in device memory (the atomics of the insertion stay on the
    // device), copied to the mailbox words afterwards
    p.vcount.reserve(2 * sizeof(int));
    HPM_HIP(hipMemsetAsync(p.vcount.p, 0, 2 * sizeof(int), s));
    a.hkeys = p.vhash_keys.as<uint32_t>();
    a.hvals = p.vhash_vals.as<int>();
    a.mask = uint32_t(slots - 1);
    a.bits = p.vhash_bits;
    k_virt_insert<<<nt, 256, 0, s>>>(a, p.vcount.as<int>(), p.vkeys.as<uint32_t>(),
                                     p.vcount.as<int>() + 1);
    HPM_LAUNCH_CHECK();
    k_copy_words<<<1, 64, 0, s>>>(p.vcount.as<int>(), p.dbox + Plan::kBoxVirt, 2);
    HPM_LAUNCH_CHECK();
    sync_box(p, s);
    if (!p.hbox[Plan::kBoxVirtFull]) {
      nv = p.hbox[Plan::kBoxVirt];
      break;
    }
    if (p.vhash_bits >= 30) fail(HPM_ERR_NO_MEMORY, "too many virtual cubes");
    p.vhash_bits += 2;
  }
  read_leaf_counts(p);
  if (nv > 0) {
    ensure_cells(p, p.ncells + nv, p.ncells, s);
    p.vlevel.reserve(size_t(nv) * 4);
    p.vlist.reserve(size_t(nv) * 4);
    k_virt_cells<<<nblk(nv, 256), 256, 0, s>>>(nv, p.vkeys.as<uint32_t>(), p.depth, int(p.n),
                                                p.keys.as<uint32_t>(), int(p.ncells),
                                                p.ccoord.as<int>(), p.cpb.as<int>(),
                                                p.cpe.as<int>(), p.vlevel.as<int>(),
                                                p.vlist.as<int>());
    HPM_LAUNCH_CHECK();
    p.nvirt = nv;
    a.coord = p.ccoord.as<int>();  // the cell arrays may have moved when they grew
    a.flags = p.cflags.as<int>();
    a.child8 = p.child8.as<int>();
    a.nbr27 = p.nbr27.as<int>();
    a.pb = p.cpb.as<int>();
    a.pe = p.cpe.as<int>();
  }
  build_block_table(p, a, nt, s);
}

}  // namespace hpm
