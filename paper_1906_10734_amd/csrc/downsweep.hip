// Down-sweep and leaves: parent-to-child translation (Sec. 2.4, Eq. 6-7), the far field at the
// particles (Eq. 7 and its gradient) and the near-zone direct sum (Sec. 1), plus a brute-force
// direct sum used as the accuracy reference.
//
// Far-field representation. A cell's local potential is kept as a constant c (a compensated pair
// of reals) plus gridlet values dPhi, Phi = c + dPhi. After source-to-target and parent-to-child
// the mean over the cell's nodes is moved into c, so dPhi holds only the variation across the
// cell. The potential is the same function; what changes is that the large potential of
// distant matter, accumulated over the levels, is never rounded together with the small
// variation from which the acceleration is differentiated.
//
// Near zone. Under the cube-complete zones a coarse leaf next to a finely refined cube of its own
// level sums over every particle in that cube, so the pair count per leaf is very uneven. The
// near-zone sources of each leaf (27 contiguous sorted ranges) are cut into chunks of kP2PChunk,
// and its targets into pieces whose sizes keep a wave's lanes busy (target_pieces); one wave
// handles one (leaf, target piece, source chunk) item and writes partial sums, and a per-leaf
// pass adds the partials in a fixed order (deterministic), adds the far field and scatters the
// results to input order.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "hpm_internal.h"

namespace hpm {

constexpr int kP2PChunk = 1024;
// Sources staged in LDS at a time: 256 in FP32; 192 in FP64, which keeps a workgroup's LDS at
// 11 KB so that two fit beside the FP64 source-to-target kernel's 133 KB on a CU.
template <typename T>
constexpr int p2p_tile() { return sizeof(T) == 4 ? 256 : 192; }
// A tile plus the pads of equal group slices: G L <= cnt + 2 G - 1 for G <= 16 (the bank skew
// below), cnt + G - 1 for G <= 64.
template <typename T>
constexpr int p2p_slots() { return p2p_tile<T>() + 64; }

// The targets of a leaf with K particles in pieces of at most 64: a wave splits its 64 lanes into
// G = floor(64 / k) groups over the sources of a k-target piece, so k in 33..55 (G = 1, at most
// 55 lanes busy) is cut as 32 + (k - 32), and 17..27 (G = 2 or 3) as 16 + (k - 16); larger leaves
// start with pieces of 64. target_piece(K, t) gives the piece of target t: its index, first target
// and size; target_pieces(K) their number.
struct Piece {
  int index, first, size;
};

__host__ __device__ __forceinline__ Piece target_piece(int K, int t) {
  const int full = (K - 1) / 64;  // leading pieces of 64
  if (t < 64 * full) return {t / 64, 64 * (t / 64), 64};
  const int r = K - 64 * full, u = t - 64 * full;
  int cut = 0;
  if (r > 32 && r < 56) cut = 32;
  else if (r > 16 && r < 28) cut = 16;
  if (cut == 0) return {full, 64 * full, r};
  return u < cut ? Piece{full, 64 * full, cut} : Piece{full + 1, 64 * full + cut, r - cut};
}

__host__ __device__ __forceinline__ int target_pieces(int K) {
  const int full = (K - 1) / 64, r = K - 64 * full;
  return full + ((r > 32 && r < 56) || (r > 16 && r < 28) ? 2 : 1);
}

template <typename T>
__device__ __forceinline__ void two_sum(T a, T b, T& s, T& e) {
  s = a + b;
  const T bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Completes the local potential of the cells of one level after source-to-target:
//   v_q = dPhi^C_q (the source-to-target result) + sum_p dPhi^P_p l_p((a^C + x_q)/2)
// (the parent's part, the transpose of the separable child-to-parent matrix; absent at level 2),
// then dPhi^C = v - mean(v) and c^C = c^P + mean(v) (+ the mean of the source-to-target result
// when that kernel delivers it apart from a zero-mean gridlet; the constant is then summed in
// double, or in float-float when that mean comes as a float pair). One workgroup per cell.
template <typename T, int NG>
__global__ __launch_bounds__(256) void k_l2l(int off, int has_parent, const int* __restrict__ parent,
                                             const int* __restrict__ coord, const T* __restrict__ t1,
                                             T* __restrict__ local, T* __restrict__ lofs,
                                             const double* __restrict__ m2l_mean, int mean_ff) {
  constexpr int M = NG * NG * NG;
  constexpr int PER = (M + 255) / 256;
  __shared__ T s_in[M], s_a[M], s_b[M];
  __shared__ T s_t[2][NG][NG];
  __shared__ T s_red[4];
  const int g = off + blockIdx.x;
  const int tid = threadIdx.x;
  const int P = has_parent ? parent[g] : -1;
  T w[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = tid + 256 * r;
    w[r] = (e < M) ? local[size_t(g) * M + e] : T(0);
  }
  if (has_parent) {
    const int pc = coord[g];
    const int ax = coord_x(pc) & 1, ay = coord_y(pc) & 1, az = coord_z(pc) & 1;
    for (int e = tid; e < 2 * NG * NG; e += 256) (&s_t[0][0][0])[e] = t1[e];
    for (int e = tid; e < M; e += 256) s_in[e] = local[size_t(P) * M + e];
    __syncthreads();
    for (int e = tid; e < M; e += 256) {  // A[pz][py][qx]
      const int qx = e % NG, rest = e / NG;
      T acc = T(0);
#pragma unroll
      for (int p = 0; p < NG; ++p) acc += s_t[ax][p][qx] * s_in[rest * NG + p];
      s_a[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < M; e += 256) {  // B[pz][qy][qx]
      const int qx = e % NG, qy = (e / NG) % NG, pz = e / (NG * NG);
      T acc = T(0);
#pragma unroll
      for (int p = 0; p < NG; ++p) acc += s_t[ay][p][qy] * s_a[(pz * NG + p) * NG + qx];
      s_b[e] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {  // out[qz][qy][qx]
      const int e = tid + 256 * r;
      if (e < M) {
        const int qx = e % NG, qy = (e / NG) % NG, qz = e / (NG * NG);
        T acc = T(0);
#pragma unroll
        for (int p = 0; p < NG; ++p) acc += s_t[az][p][qz] * s_b[(p * NG + qy) * NG + qx];
        w[r] += acc;
      }
    }
  }
  T part = T(0);
#pragma unroll
  for (int r = 0; r < PER; ++r) part += w[r];
  part = wave_sum(part);
  if ((tid & 63) == 0) s_red[tid >> 6] = part;
  __syncthreads();
  const T mean = ((s_red[0] + s_red[1]) + (s_red[2] + s_red[3])) * T(1.0 / M);
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = tid + 256 * r;
    if (e < M) local[size_t(g) * M + e] = w[r] - mean;
  }
  if (tid == 0) {
    if (m2l_mean && mean_ff) {
      // the source-to-target mean as a float pair: the constant summed in float-float
      if constexpr (sizeof(T) == 4) {
        ff32 c = ff_add(reinterpret_cast<const ff32*>(m2l_mean)[g], ff32{float(mean), 0.0f});
        if (has_parent) c = ff_add(c, ff32{float(lofs[2 * P]), float(lofs[2 * P + 1])});
        lofs[2 * g] = T(c.hi);
        lofs[2 * g + 1] = T(c.lo);
      }
    } else if (m2l_mean) {
      double c = m2l_mean[g] + double(mean);
      if (has_parent) c += double(lofs[2 * P]) + double(lofs[2 * P + 1]);
      const T hi = T(c);
      lofs[2 * g] = hi;
      lofs[2 * g + 1] = T(c - double(hi));
    } else if (has_parent) {
      T s, err;
      two_sum(lofs[2 * P], mean, s, err);
      lofs[2 * g] = s;
      lofs[2 * g + 1] = lofs[2 * P + 1] + err;
    } else {
      lofs[2 * g] = mean;
      lofs[2 * g + 1] = T(0);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Plan-time near-zone lists and the P2P work items
// ---------------------------------------------------------------------------------------------
struct NearArgs {
  int depth;
  const int* lev;  // the tree's level table (leaf count, level offsets)
  int64_t cap_cells;
  const int* leaves;
  const int* coord;
  const int* pb;
  const int* pe;
  const int* nbr27;
  const uint32_t* keys;
  int* near_rb;  // [nleaves][27]
  int* near_re;
  int* item_cnt;  // per leaf: number of work items
  int* item_off;  // their offset in the item list (within the workgroup's chunk until filled)
  int* leaf_of;   // leaf list index of each sorted particle
  unsigned long long* pairs;
  const int* vcount;  // the virtual-cube listing's words (count, full)
  int* group_items;   // per workgroup of k_near_lists: its items, then their exclusive prefix
  int* box;
};

constexpr int kNearThreads = 256;
constexpr int kNearLanes = 32;                              // lanes per leaf
constexpr int kNearPerGroup = kNearThreads / kNearLanes;   // leaves per workgroup iteration
using u64 = unsigned long long;

// 32 lanes per leaf; workgroup b takes the contiguous leaves [b L, (b+1) L), eight at a time:
// lane k < 27 finds the sorted particle range of near cube k (a real cell's range, or the part of
// a coarser leaf's range with the cube's key prefix); the lanes mark the leaf's particles with
// its list index; the leaf's targets times sources give its pairs and, cut into pieces and
// chunks, its work items. Each leaf's item offset within its workgroup's chunk goes to item_off,
// the chunk's total to group_items[b]; the item offsets are completed by k_fill_items.
__global__ __launch_bounds__(kNearThreads) void k_near_lists(NearArgs a, int per_group) {
  __shared__ int s_off[kMaxLevels + 1];
  __shared__ u64 s_pairs;
  __shared__ int s_cnt[kNearPerGroup];
  __shared__ int s_run;
  const int tid = threadIdx.x, k = tid % kNearLanes, slot = tid / kNearLanes;
  if (int64_t(a.lev[kLevCells]) > a.cap_cells) return;
  const int nl = a.lev[kLevLeaves];
  if (tid <= kMaxLevels) s_off[tid] = a.lev[kLevOff + tid];
  if (tid == 0) {
    s_pairs = 0ull;
    s_run = 0;
  }
  __syncthreads();
  u64 pairs = 0ull;
  const int first = blockIdx.x * per_group, last = min(nl, first + per_group);
  // the trip count is the same for the whole workgroup (the lane shuffles below need every lane)
  for (int base = first; base < last; base += kNearPerGroup) {
    const int li = base + slot;
    const bool live = li < last;
    const int g = live ? a.leaves[li] : 0;
    const int l = live ? level_of(g, s_off, kMaxLevels) : 0;
    int rb = 0, re = 0;
    if (live && k < 27) {
      const int e = a.nbr27[size_t(g) * 27 + k];
      if (e >= 0) {
        rb = a.pb[e];
        re = a.pe[e];
      } else if (e <= -2) {
        const int c = -2 - e;
        const int pc = a.coord[g];
        const int qx = coord_x(pc) + k % 3 - 1, qy = coord_y(pc) + (k / 3) % 3 - 1,
                  qz = coord_z(pc) + k / 9 - 1;
        const uint32_t key = morton3(uint32_t(qx), uint32_t(qy), uint32_t(qz), l);
        const int shift = 3 * (a.depth - l);
        key_range_u32(a.keys, a.pb[c], a.pe[c], key << shift, (key + 1u) << shift, rb, re);
      }
      a.near_rb[size_t(li) * 27 + k] = rb;
      a.near_re[size_t(li) * 27 + k] = re;
    }
    int S = re - rb;
#pragma unroll
    for (int o = kNearLanes / 2; o > 0; o >>= 1) S += __shfl_xor(S, o, kNearLanes);
    int items = 0;
    if (live) {
      const int b = a.pb[g], e = a.pe[g];
      for (int j = b + k; j < e; j += kNearLanes) a.leaf_of[j] = li;
      const int K = e - b;
      const int ns = (S + kP2PChunk - 1) / kP2PChunk;
      items = target_pieces(K) * max(ns, 1);
      if (k == 0) pairs += (u64)K * (u64)S;
    }
    if (k == 0) s_cnt[slot] = items;
    __syncthreads();
    if (live && k == 0) {
      int pre = s_run;
      for (int q = 0; q < slot; ++q) pre += s_cnt[q];
      a.item_cnt[li] = items;
      a.item_off[li] = pre;  // within the workgroup's chunk
    }
    __syncthreads();  // every leaf has read s_run and s_cnt
    if (tid == 0)
      for (int q = 0; q < kNearPerGroup; ++q) s_run += s_cnt[q];
    __syncthreads();
  }
  if (k == 0 && pairs) atomicAdd(&s_pairs, pairs);
  __syncthreads();
  if (tid == 0) {
    if (s_pairs) atomicAdd(a.pairs, s_pairs);
    a.group_items[blockIdx.x] = s_run;
  }
}

// One workgroup: the exclusive scan of the workgroups' item totals (their bases), the total into
// the mailbox, with the two words of the virtual-cube listing that ran before.
constexpr int kNearScanThreads = 1024;
__global__ __launch_bounds__(kNearScanThreads) void k_near_scan(NearArgs a, int groups) {
  __shared__ int s_w[kNearScanThreads / 64];
  __shared__ int s_run;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (int64_t(a.lev[kLevCells]) > a.cap_cells) return;
  if (tid == 0) s_run = 0;
  __syncthreads();
  for (int c0 = 0; c0 < groups; c0 += kNearScanThreads) {
    const int i = c0 + tid;
    const int v = i < groups ? a.group_items[i] : 0;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    int run = s_run + x - v, all = 0;
#pragma unroll
    for (int w = 0; w < kNearScanThreads / 64; ++w) {
      if (w < wave) run += s_w[w];
      all += s_w[w];
    }
    if (i < groups) a.group_items[i] = run;
    __syncthreads();  // every thread has read s_run and s_w
    if (tid == 0) s_run += all;
    __syncthreads();
  }
  if (tid == 0) {
    a.box[Plan::kBoxTotal] = s_run;
    a.box[Plan::kBoxVirt] = a.vcount[0];
    a.box[Plan::kBoxVirtFull] = a.vcount[1];
  }
}

// Completes each leaf's item offset (its workgroup's base plus its offset within the chunk) and
// writes its work items.
__global__ void k_fill_items(int nleaves, int per_group, const int* group_base, int* item_off,
                             const int* pb, const int* pe, const int* leaves, const int* near_rb,
                             const int* near_re, int4* items) {
  const int li = blockIdx.x * blockDim.x + threadIdx.x;
  if (li >= nleaves) return;
  int S = 0;
  for (int k = 0; k < 27; ++k) S += near_re[li * 27 + k] - near_rb[li * 27 + k];
  const int g = leaves[li];
  const int K = pe[g] - pb[g];
  const int ns = max((S + kP2PChunk - 1) / kP2PChunk, 1);
  int it = group_base[li / per_group] + item_off[li];
  item_off[li] = it;
  for (int t = 0; t < K;) {
    const Piece pc = target_piece(K, t);
    for (int sc = 0; sc < ns; ++sc) items[it++] = make_int4(li, pc.first, pc.size, sc * kP2PChunk);
    t = pc.first + pc.size;
  }
}

static inline int nblk(int64_t n, int t) { return int((n + t - 1) / t); }

void enqueue_near_lists(Plan& p, hipStream_t s) {
  const size_t cap = size_t(p.cap_cells);  // leaves <= cells <= capacity
  p.near_rb.reserve(cap * 27 * 4);
  p.near_re.reserve(cap * 27 * 4);
  p.item_cnt.reserve(cap * 4);
  p.item_off.reserve(cap * 4);
  p.leaf_of.reserve(size_t(std::max<int64_t>(p.n, 1)) * 4);
  NearArgs a;
  a.depth = p.depth;
  a.lev = p.dlev.as<int>();
  a.cap_cells = p.cap_cells;
  a.leaves = p.leaves.as<int>();
  a.coord = p.ccoord.as<int>();
  a.pb = p.cpb.as<int>();
  a.pe = p.cpe.as<int>();
  a.nbr27 = p.nbr27.as<int>();
  a.keys = p.keys.as<uint32_t>();
  a.near_rb = p.near_rb.as<int>();
  a.near_re = p.near_re.as<int>();
  a.item_cnt = p.item_cnt.as<int>();
  a.item_off = p.item_off.as<int>();
  a.leaf_of = p.leaf_of.as<int>();
  a.pairs = p.pairs.as<unsigned long long>();
  a.vcount = p.vcount.as<int>();
  // contiguous chunks of leaves per workgroup, sized for the capacity (the leaf count is read on
  // the device): at most 16384 workgroups, at least 8 leaves each
  const int per = std::max<int>(kNearPerGroup, int(nblk(int64_t(cap), 16384)));
  p.near_per_group = (per + kNearPerGroup - 1) / kNearPerGroup * kNearPerGroup;
  p.near_groups = std::max(1, nblk(int64_t(cap), p.near_per_group));
  p.near_group_items.reserve(size_t(p.near_groups) * 4);
  a.group_items = p.near_group_items.as<int>();
  a.box = p.dbox;
  k_near_lists<<<p.near_groups, kNearThreads, 0, s>>>(a, p.near_per_group);
  HPM_LAUNCH_CHECK();
  k_near_scan<<<1, kNearScanThreads, 0, s>>>(a, p.near_groups);
  HPM_LAUNCH_CHECK();
}

void finish_near_lists(Plan& p, hipStream_t s) {
  const int nl = int(p.nleaves);
  const int total = int(p.n_items);
  p.p2p_pairs = -1;  // read from the device on request
  p.items.reserve(size_t(std::max(total, 1)) * sizeof(int4));
  p.partial.reserve(size_t(std::max(total, 1)) * 64 * 5 * p.elem);
  if (nl <= 0) return;
  k_fill_items<<<nblk(nl, 256), 256, 0, s>>>(nl, p.near_per_group, p.near_group_items.as<int>(),
                                             p.item_off.as<int>(), p.cpb.as<int>(),
                                             p.cpe.as<int>(), p.leaves.as<int>(),
                                             p.near_rb.as<int>(), p.near_re.as<int>(),
                                             p.items.as<int4>());
  HPM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------------------------
// Near zone: one wave per work item
// ---------------------------------------------------------------------------------------------
template <typename T>
struct P2PArgs {
  const int4* items;
  const int* leaves;
  const int* pb;
  const int* pe;
  const int* near_rb;
  const int* near_re;
  const T* xs;
  const T* ys;
  const T* zs;
  const T* ms;
  T* partial;  // [item][64][5]: phi, phi compensation, ax, ay, az (without G)
  T eps2;
  T inv_lam;  // 1 / screening length (screened kernel)
  T padx, pady, padz;  // a point outside the root cell (box_lo - box_size on each axis)
};

// 1/sqrt(x). In single precision the hardware reciprocal square root (about 1 ulp); the softened
// squared distances it sees are far above the denormal range, so no input scaling is needed.
// In double: the hardware's estimate refined by two Newton-Raphson steps for f(y) = 1/y^2 - x,
// y <- y + y (1 - x y^2) / 2; each step squares the relative error, which leaves it at
// rounding level. x = 0 keeps the estimate (+inf).
template <typename T>
__device__ __forceinline__ T inv_sqrt(T x) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_amdgcn_rsqf(x);
  } else {
    double y = __builtin_amdgcn_rsq(x);
    if (!(x > 0.0) || isinf(x)) return y;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const double e = fma(-x * y, y, 1.0);
      y = fma(0.5 * y, e, y);
    }
    return y;
  }
}

// Pair terms of the interaction kernel (without G) from inv = 1/s, s the softened distance:
// the potential of a unit source is -w and its acceleration -c (r_i - r_j).
//   HPM_KERNEL_NEWTON  w = 1/s,                c = 1/s^3
//   HPM_KERNEL_YUKAWA  w = exp(-s/lam)/s,      c = exp(-s/lam) (1/(lam s^2) + 1/s^3)
// inv = 0 (the self pair) gives w = c = 0 for both.
template <int KER, typename T>
__device__ __forceinline__ void pair_terms(T s2, T inv, T inv_lam, T& w, T& c) {
  if constexpr (KER == HPM_KERNEL_NEWTON) {
    w = inv;
    c = inv * inv * inv;
  } else {
    const T e = exp(-(s2 * inv) * inv_lam);
    w = e * inv;
    c = w * (inv * inv + inv * inv_lam);
  }
}

template <typename T>
struct alignas(4 * sizeof(T)) SrcP {
  T x, y, z, m;
};

// Element j of a particle array. Single precision addresses it with a 32-bit byte offset
// (n <= 2^30), which lets the load take the array base from scalar registers.
template <typename T>
__device__ __forceinline__ T load_at(const T* base, int j) {
  if constexpr (sizeof(T) == 4) {
    const uint32_t off = uint32_t(j) << 2;
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
  } else {
    return base[uint32_t(j)];
  }
}

// Item (leaf, first target t0, piece size kp, first source s0): lanes split as (target tl < kp,
// source group grp < G = 64/kp) (lanes past the last whole group idle). Sources are staged
// p2p_tile at a time in LDS (position and mass in one 4-vector). Each group takes L =
// ceil(cnt / G) of a tile's cnt sources, so every lane runs the same trip count: in FP32 the
// contiguous slice [grp L, grp L + L), in FP64 the slots grp, grp + G, ... The slots past cnt
// hold massless sources at a point outside the root cell: their pair terms are finite and their
// products with the zero mass are exact zeros, so they change no sum. For FP32 slices and
// G <= 16, L is bumped off multiples of 8 so that two groups' 16-byte reads in one LDS pass fall
// in different banks. Each lane sums a tile's pair potentials in plain arithmetic and adds the
// tile's sum to its running total with compensation (Kahan); the groups' partial sums are
// combined in group order through LDS. The self pair is recognised by its place in the source
// sequence: the target leaf's own cube is entry 13 of its 27 near cubes.
template <typename T, int KER>
__global__ __launch_bounds__(64) void k_p2p(P2PArgs<T> a) {
  __shared__ int s_rb[27], s_pre[28];
  constexpr int kTile = p2p_tile<T>(), kSlots = p2p_slots<T>();
  __shared__ SrcP<T> s_src[kSlots];
  __shared__ T s_part[5][64];
  const int lane = threadIdx.x;
  const int4 it = a.items[blockIdx.x];
  const int li = it.x, t0 = it.y, kp = it.z, s0 = it.w;
  const int g = a.leaves[li];
  const int pb = a.pb[g];
  if (lane < 27) s_rb[lane] = a.near_rb[li * 27 + lane];
  {
    const int len = (lane < 27) ? a.near_re[li * 27 + lane] - a.near_rb[li * 27 + lane] : 0;
    int x = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane < 28) s_pre[lane] = x - len;  // exclusive prefix; s_pre[27] = total
  }
  __syncthreads();
  const int S = s_pre[27];
  // FP32 reads group slices (immediate LDS offsets); FP64 reads the groups' sources interleaved,
  // whose 32-byte reads of one pass are contiguous and so never share a bank.
  constexpr bool kSlices = sizeof(T) == 4;
  const int G = 64 / kp;
  const int tl = lane % kp, grp = lane / kp;
  const int i = pb + t0 + tl;
  const bool valid = grp < G;
  const int self = s_pre[13] + (i - s_rb[13]);  // the target's own place in the source sequence
  T xi = T(0), yi = T(0), zi = T(0);
  if (valid) {
    xi = a.xs[i];
    yi = a.ys[i];
    zi = a.zs[i];
  }
  T ph = T(0), phc = T(0), fx = T(0), fy = T(0), fz = T(0);
  const int s_end = min(S, s0 + kP2PChunk);
  // the piece's own targets occupy [self_lo, self_hi) of the source sequence
  const int self_lo = s_pre[13] + (pb + t0 - s_rb[13]), self_hi = self_lo + kp;
  // Staging cursor: the near cube r holding this lane's next source (the largest r with
  // s_pre[r] <= source). A lane's sources only increase, so r only moves forward.
  int r = 0;
  {
    const int first = min(s0 + lane, S - 1);
    int hi = 27;
    while (hi - r > 1) {
      const int mid = (r + hi) >> 1;
      if (s_pre[mid] <= first) r = mid;
      else hi = mid;
    }
  }
  T pt = T(0);  // potential of the current tile
  auto pair = [&](const SrcP<T>& q, bool skip) {
    const T dx = xi - q.x, dy = yi - q.y, dz = zi - q.z;
    const T r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, a.eps2)));
    const T inv = skip ? T(0) : inv_sqrt(r2);
    T w, c;
    pair_terms<KER>(r2, inv, a.inv_lam, w, c);
    const T mi3 = q.m * c;
    pt = fma(-q.m, w, pt);
    fx = fma(-mi3, dx, fx);
    fy = fma(-mi3, dy, fy);
    fz = fma(-mi3, dz, fz);
  };
  for (int tile = s0; tile < s_end; tile += kTile) {
    const int cnt = min(kTile, s_end - tile);
    int L = (cnt + G - 1) / G;
    if (kSlices && G <= 16 && (L & 7) == 0) ++L;
    const int slots = G * L;  // <= kSlots
    // FP32 has all loads of the tile in flight before the first LDS write. FP64 stages one slot
    // per lane at a time: that keeps the kernel within the 104 VGPRs per SIMD lane that the FP64
    // source-to-target kernel (406 per wave) leaves free, so the two can share a SIMD when the
    // near zone runs beside it.
    constexpr int kStage = kSlots / 64;
    constexpr int kBatch = sizeof(T) == 4 ? kStage : 1;
    if (kBatch < kStage) __syncthreads();  // the previous tile's reads are done
    for (int k0 = 0; k0 < kStage; k0 += kBatch) {
      SrcP<T> v[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int q = lane + 64 * (k0 + k);
        v[k] = SrcP<T>{a.padx, a.pady, a.padz, T(0)};
        if (q < cnt) {
          const int sidx = tile + q;
          while (s_pre[r + 1] <= sidx) ++r;  // s_pre[27] = S > sidx ends it
          const int j = s_rb[r] + (sidx - s_pre[r]);
          v[k] = SrcP<T>{load_at(a.xs, j), load_at(a.ys, j), load_at(a.zs, j), load_at(a.ms, j)};
        }
      }
      if (kBatch == kStage) __syncthreads();  // the previous tile's reads are done
#pragma unroll
      for (int k = 0; k < kBatch; ++k)
        if (lane + 64 * (k0 + k) < slots) s_src[lane + 64 * (k0 + k)] = v[k];
    }
    __syncthreads();
    if (valid) {
      // this group's e-th source: slot grp L + e (slices) or grp + e G (interleaved)
      const SrcP<T>* src = s_src + (kSlices ? grp * L : grp);
      const int step = kSlices ? 1 : G;
      pt = T(0);
      if (tile < self_hi && tile + cnt > self_lo) {  // the tile may hold the target itself
        const int own = self - tile;                 // the target's slot in the tile
        for (int e = 0; e < L; ++e) pair(src[e * step], (kSlices ? grp * L + e : grp + e * G) == own);
      } else {
#pragma unroll 4
        for (int e = 0; e < L; ++e) pair(src[e * step], false);
      }
      const T yv = pt - phc;  // Kahan: ph += pt
      const T tv = ph + yv;
      phc = (tv - ph) - yv;
      ph = tv;
    }
  }
  if (G > 1) {
    s_part[0][lane] = ph;
    s_part[1][lane] = -phc;
    s_part[2][lane] = fx;
    s_part[3][lane] = fy;
    s_part[4][lane] = fz;
  }
  __syncthreads();
  if (grp == 0) {
    T phs = ph, phe = -phc;
    for (int q = 1; q < G; ++q) {
      const int o = q * kp + tl;
      T s, err;
      two_sum(phs, s_part[0][o], s, err);
      phe += s_part[1][o] + err;
      phs = s;
      fx += s_part[2][o];
      fy += s_part[3][o];
      fz += s_part[4][o];
    }
    T* out = a.partial + (size_t(blockIdx.x) * 64 + tl) * 5;
    out[0] = phs;
    out[1] = phe;
    out[2] = fx;
    out[3] = fy;
    out[4] = fz;
  }
}

// ---------------------------------------------------------------------------------------------
// Per leaf: add the partials, the far field (Eq. 7 and its gradient), scatter to input order
// ---------------------------------------------------------------------------------------------
template <typename T>
struct LeafArgs {
  int n;
  const int* leaves;
  const int* level_off;
  int nlevels;
  const int* coord;
  const int* pb;
  const int* pe;
  const int* item_off;
  const int* item_cnt;
  const int* leaf_of;  // leaf list index of each sorted particle
  const int* perm;
  const T* xs;
  const T* ys;
  const T* zs;
  const T* local;
  const T* lofs;
  const T* partial;
  T* phi;
  T* ax;
  T* ay;
  T* az;
  double lo0, lo1, lo2, size;
  T gconst;
};

// One lane per sorted particle: workgroup b takes particles [64 b, 64 b + 64). They belong to a
// few leaves (runs of consecutive particles), whose local potentials are staged in LDS kLeafRuns
// at a time; a lane's near-zone partials are found from its place in its leaf. The local
// potential lives on NP = N_g + 2 EXT nodes per axis (EXT = 1: the extended gridlet of Sec. 2.5).
constexpr int kLeafRuns = 4;

template <typename T, int NG, int EXT>
__global__ __launch_bounds__(64) void k_leaf(LeafArgs<T> a) {
  constexpr int NP = NG + 2 * EXT;
  constexpr int M = NP * NP * NP;
  __shared__ int s_off[kMaxLevels + 1];
  __shared__ int s_run_leaf[64];
  __shared__ T s_phi[kLeafRuns][M];
  const int lane = threadIdx.x;
  if (lane <= kMaxLevels) s_off[lane] = a.level_off[lane];
  const int i = blockIdx.x * 64 + lane;
  const int li = i < a.n ? a.leaf_of[i] : -1;  // -1: past the end (or in no leaf)
  const bool valid = li >= 0;
  const int prev = __shfl_up(li, 1, 64);
  const bool start = valid && (lane == 0 || prev != li);
  const uint64_t starts = __ballot(start);
  const int run = __popcll(starts & ((2ull << lane) - 1ull)) - 1;  // run of this lane
  const int nruns = __popcll(starts);
  if (start) s_run_leaf[run] = li;
  __syncthreads();

  int g = 0, l = 0, pb = 0, K = 1, pc = 0;
  if (valid) {
    g = a.leaves[li];
    l = level_of(g, s_off, a.nlevels);
    pb = a.pb[g];
    K = a.pe[g] - pb;
    pc = a.coord[g];
  }
  const double L = a.size / double(1 << l);
  const T invL = T(1.0 / L);
  // near zone: partials of this particle's target chunk, source chunks in order
  T ph = T(0), phe = T(0), fx = T(0), fy = T(0), fz = T(0);
  if (valid) {
    const int t = i - pb;
    const Piece pc = target_piece(K, t);
    const int ns = a.item_cnt[li] / target_pieces(K);
    for (int sc = 0; sc < ns; ++sc) {
      const T* q = a.partial + (size_t(a.item_off[li] + pc.index * ns + sc) * 64 + (t - pc.first)) * 5;
      T s, err;
      two_sum(ph, q[0], s, err);
      ph = s;
      phe += q[1] + err;
      fx += q[2];
      fy += q[3];
      fz += q[4];
    }
  }
  // far field from c + dPhi, the leaves' potentials staged kLeafRuns at a time
  T pfar = T(0), gx = T(0), gy = T(0), gz = T(0);
  for (int r0 = 0; r0 < nruns; r0 += kLeafRuns) {
    __syncthreads();  // the previous round's gridlets are consumed
    for (int q = 0; q < kLeafRuns && r0 + q < nruns; ++q) {
      const int gq = a.leaves[s_run_leaf[r0 + q]];
      if (level_of(gq, s_off, a.nlevels) >= 2)
        for (int e = lane; e < M; e += 64) s_phi[q][e] = a.local[size_t(gq) * M + e];
    }
    __syncthreads();
    if (valid && l >= 2 && run >= r0 && run < r0 + kLeafRuns) {
      const T* phi = s_phi[run - r0];
      const T cxc = T(a.lo0 + (coord_x(pc) + 0.5) * L), cyc = T(a.lo1 + (coord_y(pc) + 0.5) * L),
              czc = T(a.lo2 + (coord_z(pc) + 0.5) * L);
      const T xi = a.xs[i], yi = a.ys[i], zi = a.zs[i];
      T lx[NP], dlx[NP], ly[NP], dly[NP], lz[NP], dlz[NP];
      lagrange_basis_d<NG, EXT>((xi - cxc) * invL, lx, dlx);
      lagrange_basis_d<NG, EXT>((yi - cyc) * invL, ly, dly);
      lagrange_basis_d<NG, EXT>((zi - czc) * invL, lz, dlz);
#pragma unroll
      for (int k = 0; k < NP; ++k) {
#pragma unroll
        for (int j = 0; j < NP; ++j) {
          T r0v = T(0), r1v = T(0);
#pragma unroll
          for (int q = 0; q < NP; ++q) {
            const T v = phi[(k * NP + j) * NP + q];
            r0v += lx[q] * v;
            r1v += dlx[q] * v;
          }
          pfar += lz[k] * ly[j] * r0v;
          gx += lz[k] * ly[j] * r1v;
          gy += lz[k] * dly[j] * r0v;
          gz += dlz[k] * ly[j] * r0v;
        }
      }
    }
  }
  if (!valid) return;
  // phi = G*near + c + dPhi(x), added with compensation
  const T c_hi = (l >= 2) ? a.lofs[2 * g] : T(0), c_lo = (l >= 2) ? a.lofs[2 * g + 1] : T(0);
  const T gn = a.gconst;
  const T n_hi = gn * ph;
  const T n_lo = fma(gn, ph, -n_hi) + gn * phe;
  T s1, e1, s2, e2;
  two_sum(n_hi, c_hi, s1, e1);
  two_sum(s1, pfar, s2, e2);
  const int o = a.perm[i];
  if (o < 0 || o >= a.n) return;
  a.phi[o] = s2 + (e2 + (e1 + (n_lo + c_lo)));
  a.ax[o] = gn * fx - gx * invL;
  a.ay[o] = gn * fy - gy * invL;
  a.az[o] = gn * fz - gz * invL;
}

template <typename T, int KER>
__global__ __launch_bounds__(256) void k_direct(int n, const T* x, const T* y, const T* z, const T* m,
                                                const int* targets, double G, double eps2,
                                                double inv_lam, double* phi, double* ax, double* ay,
                                                double* az) {
  __shared__ double s_red[4][4];
  const int t = targets[blockIdx.x];
  if (t < 0 || t >= n) {  // invalid target index: NaN result, no out-of-range read
    if (threadIdx.x == 0) phi[blockIdx.x] = ax[blockIdx.x] = ay[blockIdx.x] = az[blockIdx.x] = __builtin_nan("");
    return;
  }
  const double xi = x[t], yi = y[t], zi = z[t];
  double p = 0, fx = 0, fy = 0, fz = 0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    if (j == t) continue;
    const double dx = xi - double(x[j]), dy = yi - double(y[j]), dz = zi - double(z[j]);
    const double r2 = dx * dx + dy * dy + dz * dz + eps2;
    const double inv = 1.0 / sqrt(r2);
    double w, c;
    pair_terms<KER>(r2, inv, inv_lam, w, c);
    const double mi = double(m[j]) * w;
    const double mi3 = double(m[j]) * c;
    p -= mi;
    fx -= mi3 * dx;
    fy -= mi3 * dy;
    fz -= mi3 * dz;
  }
  p = wave_sum(p);
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  fz = wave_sum(fz);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_red[w][0] = p;
    s_red[w][1] = fx;
    s_red[w][2] = fy;
    s_red[w][3] = fz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k)
      for (int v = 0; v < 4; ++v) r[v] += s_red[k][v];
    phi[blockIdx.x] = G * r[0];
    ax[blockIdx.x] = G * r[1];
    ay[blockIdx.x] = G * r[2];
    az[blockIdx.x] = G * r[3];
  }
}

template <typename T, int NG>
static void l2l_t(Plan& p, int level, hipStream_t s) {
  const int off = p.level_off[level];
  const int cnt = p.level_off[level + 1] - off;
  if (cnt <= 0) return;
  k_l2l<T, NG><<<cnt, 256, 0, s>>>(off, level >= 3 ? 1 : 0, p.cparent.as<int>(), p.ccoord.as<int>(),
                                   p.tab.l2l.as<T>(), p.local.as<T>(), p.lofs.as<T>(),
                                   p.m2l_split ? p.m2l_mean.as<double>() : nullptr,
                                   p.m2l_mean_ff ? 1 : 0);
  HPM_LAUNCH_CHECK();
}

template <typename T>
static void p2p_t(Plan& p, hipStream_t s) {
  if (p.nleaves <= 0 || p.n_items <= 0) return;
  P2PArgs<T> b;
  b.items = p.items.as<int4>();
  b.leaves = p.leaves.as<int>();
  b.pb = p.cpb.as<int>();
  b.pe = p.cpe.as<int>();
  b.near_rb = p.near_rb.as<int>();
  b.near_re = p.near_re.as<int>();
  b.xs = p.xs.as<T>();
  b.ys = p.ys.as<T>();
  b.zs = p.zs.as<T>();
  b.ms = p.ms.as<T>();
  b.partial = p.partial.as<T>();
  b.eps2 = T(p.prob.softening * p.prob.softening);
  b.inv_lam = (p.prob.kernel == HPM_KERNEL_YUKAWA) ? T(1.0 / p.prob.screening) : T(0);
  b.padx = T(p.prob.box_lo[0] - p.prob.box_size);
  b.pady = T(p.prob.box_lo[1] - p.prob.box_size);
  b.padz = T(p.prob.box_lo[2] - p.prob.box_size);
  if (p.prob.kernel == HPM_KERNEL_YUKAWA) k_p2p<T, HPM_KERNEL_YUKAWA><<<int(p.n_items), 64, 0, s>>>(b);
  else k_p2p<T, HPM_KERNEL_NEWTON><<<int(p.n_items), 64, 0, s>>>(b);
  HPM_LAUNCH_CHECK();
}

template <typename T, int NG, int EXT>
static void leaf_t(Plan& p, void* phi, void* ax, void* ay, void* az, hipStream_t s) {
  if (p.nleaves <= 0 || p.n_items <= 0) return;
  LeafArgs<T> a;
  a.n = int(p.n);
  a.leaves = p.leaves.as<int>();
  a.level_off = p.dlev.as<int>() + kLevOff;
  a.nlevels = p.nlevels;
  a.coord = p.ccoord.as<int>();
  a.pb = p.cpb.as<int>();
  a.pe = p.cpe.as<int>();
  a.item_off = p.item_off.as<int>();
  a.item_cnt = p.item_cnt.as<int>();
  a.leaf_of = p.leaf_of.as<int>();
  a.perm = p.perm.as<int>();
  a.xs = p.xs.as<T>();
  a.ys = p.ys.as<T>();
  a.zs = p.zs.as<T>();
  a.local = p.local.as<T>();
  a.lofs = p.lofs.as<T>();
  a.partial = p.partial.as<T>();
  a.phi = (T*)phi;
  a.ax = (T*)ax;
  a.ay = (T*)ay;
  a.az = (T*)az;
  a.lo0 = p.prob.box_lo[0];
  a.lo1 = p.prob.box_lo[1];
  a.lo2 = p.prob.box_lo[2];
  a.size = p.prob.box_size;
  a.gconst = T(p.prob.gconst);
  k_leaf<T, NG, EXT><<<nblk(p.n, 64), 64, 0, s>>>(a);
  HPM_LAUNCH_CHECK();
}

// parent-to-child runs on the target gridlet's NL = N_g + 2 ext nodes per axis
void launch_l2l(Plan& p, int level, hipStream_t s) {
  if (p.prec == HPM_F32) {
    switch (p.NL) {
      case 2: l2l_t<float, 2>(p, level, s); break;
      case 3: l2l_t<float, 3>(p, level, s); break;
      case 4: l2l_t<float, 4>(p, level, s); break;
      case 5: l2l_t<float, 5>(p, level, s); break;
      case 6: l2l_t<float, 6>(p, level, s); break;
      case 8: l2l_t<float, 8>(p, level, s); break;
      default: fail(HPM_ERR_UNSUPPORTED, "no parent-to-child kernel for this gridlet");
    }
  } else {
    switch (p.NL) {
      case 2: l2l_t<double, 2>(p, level, s); break;
      case 3: l2l_t<double, 3>(p, level, s); break;
      case 4: l2l_t<double, 4>(p, level, s); break;
      case 5: l2l_t<double, 5>(p, level, s); break;
      case 6: l2l_t<double, 6>(p, level, s); break;
      case 8: l2l_t<double, 8>(p, level, s); break;
      default: fail(HPM_ERR_UNSUPPORTED, "no parent-to-child kernel for this gridlet");
    }
  }
}

template <typename T>
static void leaf_dispatch(Plan& p, void* phi, void* ax, void* ay, void* az, hipStream_t s) {
  const int key = p.ng * 2 + p.ext;
  switch (key) {
    case 4: leaf_t<T, 2, 0>(p, phi, ax, ay, az, s); break;
    case 5: leaf_t<T, 2, 1>(p, phi, ax, ay, az, s); break;
    case 6: leaf_t<T, 3, 0>(p, phi, ax, ay, az, s); break;
    case 7: leaf_t<T, 3, 1>(p, phi, ax, ay, az, s); break;
    case 8: leaf_t<T, 4, 0>(p, phi, ax, ay, az, s); break;
    case 9: leaf_t<T, 4, 1>(p, phi, ax, ay, az, s); break;
    case 12: leaf_t<T, 6, 0>(p, phi, ax, ay, az, s); break;
    case 13: leaf_t<T, 6, 1>(p, phi, ax, ay, az, s); break;
    case 16: leaf_t<T, 8, 0>(p, phi, ax, ay, az, s); break;
    default: fail(HPM_ERR_UNSUPPORTED, "no leaf kernel for this gridlet");
  }
}

void launch_p2p(Plan& p, hipStream_t s) {
  if (p.prec == HPM_F32) p2p_t<float>(p, s);
  else p2p_t<double>(p, s);
}

void launch_leaf(Plan& p, void* phi, void* ax, void* ay, void* az, hipStream_t s) {
  if (p.prec == HPM_F32) leaf_dispatch<float>(p, phi, ax, ay, az, s);
  else leaf_dispatch<double>(p, phi, ax, ay, az, s);
}

template <typename T>
static void direct_t(int64_t n, const void* x, const void* y, const void* z, const void* m,
                     int64_t nt, const int32_t* targets, double G, double eps, PairKernel ker,
                     double* phi, double* ax, double* ay, double* az, hipStream_t s) {
  const double inv_lam = (ker.kind == HPM_KERNEL_YUKAWA) ? 1.0 / ker.screening : 0.0;
  if (ker.kind == HPM_KERNEL_YUKAWA)
    k_direct<T, HPM_KERNEL_YUKAWA><<<int(nt), 256, 0, s>>>(int(n), (const T*)x, (const T*)y,
                                                           (const T*)z, (const T*)m, targets, G,
                                                           eps * eps, inv_lam, phi, ax, ay, az);
  else
    k_direct<T, HPM_KERNEL_NEWTON><<<int(nt), 256, 0, s>>>(int(n), (const T*)x, (const T*)y,
                                                           (const T*)z, (const T*)m, targets, G,
                                                           eps * eps, inv_lam, phi, ax, ay, az);
  HPM_LAUNCH_CHECK();
}

void launch_direct_sum(int prec, int64_t n, const void* x, const void* y, const void* z,
                       const void* m, int64_t nt, const int32_t* targets, double G, double eps,
                       PairKernel ker, double* phi, double* ax, double* ay, double* az,
                       hipStream_t s) {
  if (nt <= 0) return;
  if (prec == HPM_F32) direct_t<float>(n, x, y, z, m, nt, targets, G, eps, ker, phi, ax, ay, az, s);
  else direct_t<double>(n, x, y, z, m, nt, targets, G, eps, ker, phi, ax, ay, az, s);
}

}  // namespace hpm
