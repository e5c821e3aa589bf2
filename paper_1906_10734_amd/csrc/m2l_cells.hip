// Source-to-target (M2L) cell by cell: the alternative to the single padded grid that the paper
// weighs and sets aside (Sec. 2.5). It computes the same sums as the (8 N_g)^3 route: every
// target node receives G(target node - source node) times each effective mass of its 189
// interaction-zone cubes (Sec. 2.1, Eq. 1).
//
// Each source cube's gridlet, zero padded to C^3 with C = 2 N_g, is transformed once per solve.
// For a target and one of its sources at cube offset d = source - target (|d|_inf in 2..3), the
// C^3 cyclic array whose entry u holds g(h |d N_g - u_c|), where u_c = u for u < N_g and
// u - C otherwise, convolved cyclically with the padded source gives the potential at the
// target's N_g^3 nodes in the corner [0, N_g)^3: every node offset d N_g + (p - q) of the pair,
// |p - q| < N_g per axis, lands on a distinct entry, so nothing wraps. The transforms of these
// arrays (one per offset and level, divided by C^3) are constant tables. The sum over sources is
// taken in frequency space, then one pruned inverse transform per target keeps the corner.
//
// The paper's operation count charges one padded transform per (target, source) pair; here a
// source's transform is shared by every target that sees it (up to 27 parents' blocks), so what
// remains per pair is the pointwise product, C^2 (N_g + 1) complex multiply-adds.
//
// Kernels:
//   k_cells_forward   one wave per source gridlet (cells of levels >= 2 and virtual cubes):
//                     half spectrum [kz < C][ky < C][kx <= N_g] by separable direct sums.
//   k_cells_accum     one thread per (parent, mode), one launch per parent level. The Green table
//                     of the level is shared by every parent, so a workgroup stages its chunk of
//                     modes in LDS and runs several parents side by side; the 8 children of a
//                     parent share the 6^3 block of sources, so for each source plane bz a
//                     thread keeps that plane's 36 spectra in registers and applies each Green
//                     entry to every child and slot it joins (up to 4 of them). Only the split
//                     parents are visited, from a list built with the tree.
//   k_cells_inverse   one workgroup per target: pruned inverse (z, then y, then the Hermitian x
//                     sum), the N_g^3 corner written as the target's gridlet potentials. The
//                     inverse runs in double whatever the plan's precision (it is a small part of
//                     the work); in FP32 plans the result is stored as its mean (double) plus the
//                     zero-mean gridlet, so that the large common value of a target's potentials
//                     does not cost the precision of their differences.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "fft.h"
#include "hpm_internal.h"

#include <algorithm>

namespace hpm {

// EXT = 1: extended target gridlets (N_g + 2 nodes per axis, Sec. 2.5). Target-minus-source
// node offsets then span 2 N_g + 1 values per axis, and C = 2 N_g + 2 keeps them apart.
template <int NG, int EXT>
struct CellShape {
  static constexpr int C = 2 * NG + 2 * EXT;
  static constexpr int HC = C / 2 + 1;
  static constexpr int K = C * C * HC;      // modes, [kz][ky][kx]
  static constexpr int KP = (K + 15) / 16 * 16;  // stored row: K modes, then zeros
  static constexpr int M = NG * NG * NG;    // source gridlet
  static constexpr int NL = NG + 2 * EXT;   // target gridlet nodes per axis
  static constexpr int ML = NL * NL * NL;
  static constexpr int OFFS = 343;          // d in [-3, 3]^3, index (dx+3) + 7 (dy+3) + 49 (dz+3)
};

// e^{sign 2 pi i j / C} for j < C, in LDS (double sincospi, rounded once to T)
template <typename T, int C>
__device__ __forceinline__ void load_twiddles(cplx<T>* tw, double sign) {
  const int j = threadIdx.x;
  if (j < C) {
    double s, c;
    sincospi(2.0 * j / C, &s, &c);
    tw[j] = {T(c), T(sign * s)};
  }
}

template <typename T>
struct CellArgs {
  int first_cell;    // id of the first cell of level 2: sources and targets are indexed from it
  int nsources;      // cells of levels >= 2, then the virtual cubes (row nsources of the
                     // source spectra is zero)
  int first_parent;  // first row of the block table (cells of level 1)
  int nlevels;
  const int* level_off;
  const int* child8;
  const int* blocks;
  const T* gridlet;
  T* local;
  const cplx<T>* gcell;  // [level - 2][343][K]
  cplx<T>* sspec;        // [source - first_cell][K]
  cplx<T>* tspec;        // [target - first_cell][K]
  double* m2l_mean;      // [cells]: mean of each target's result, FP32 plans
};

// One wave per source (kFwdSources per workgroup; packing four measured slower than one). Each
// pass gives every
// lane whole lines: a lane loads the N_g nonzero samples of its line into registers and forms
// all the line's outputs with compile-time twiddles (exp(-2 pi i jk / C) as immediates), so no
// output waits on a chain of table loads. Sums run over the samples in order, as the separable
// definition reads.
constexpr int kFwdSources = 1;
constexpr int kFwdThreads = 64 * kFwdSources;

// out[k] = sum_j v[j] w^{jk}, w = exp(-2 pi i / C), for the K outputs of one line
template <typename T, int NG, int C, int K, bool REAL_IN>
__device__ __forceinline__ void line_dft(const cplx<T> (&v)[NG], cplx<T>* out, int stride) {
  static_for<0, K>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    cplx<T> acc = {T(0), T(0)};
    static_for<0, NG>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      constexpr T wr = T(cis_cos(long(j) * k, C)), wi = T(-cis_sin(long(j) * k, C));
      if constexpr (REAL_IN) {
        acc.re += v[j].re * wr;
        acc.im += v[j].re * wi;
      } else {
        acc = cadd(acc, cmul(v[j], cplx<T>{wr, wi}));
      }
    });
    out[k * stride] = acc;
  });
}

template <typename T, int NG, int EXT>
__global__ __launch_bounds__(kFwdThreads) void k_cells_forward(CellArgs<T> a) {
  using S = CellShape<NG, EXT>;
  constexpr int C = S::C, HC = S::HC, K = S::K, KP = S::KP, M = S::M;
  __shared__ T s_gw[kFwdSources][M];
  __shared__ cplx<T> s_a1w[kFwdSources][NG * NG * HC];  // [z][y][kx]
  __shared__ cplx<T> s_a2w[kFwdSources][NG * C * HC];   // [z][ky][kx]
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int src = blockIdx.x * kFwdSources + wave;
  // every wave passes every barrier; only waves with a source of their own do its work
  const bool zero_row = src == a.nsources, work = src < a.nsources;
  T* s_g = s_gw[wave];
  cplx<T>* s_a1 = s_a1w[wave];
  cplx<T>* s_a2 = s_a2w[wave];
  cplx<T>* out = a.sspec + size_t(src) * KP;
  if (zero_row)  // the zero row that empty block slots read
    for (int e = lane; e < KP; e += 64) out[e] = {T(0), T(0)};
  if (work) {
    const T* g = a.gridlet + size_t(a.first_cell + src) * M;
    for (int e = lane; e < M; e += 64) s_g[e] = g[e];
  }
  __syncthreads();
  // x: one real row (z, y) per lane, its half spectrum kx <= C/2
  if (work) {
    for (int r = lane; r < NG * NG; r += 64) {
      cplx<T> v[NG];
#pragma unroll
      for (int x = 0; x < NG; ++x) v[x] = {s_g[r * NG + x], T(0)};
      line_dft<T, NG, C, HC, true>(v, s_a1 + r * HC, 1);
    }
  }
  __syncthreads();
  // y: one column (z, kx) per lane, all C values of ky
  if (work) {
    for (int q = lane; q < NG * HC; q += 64) {
      const int z = q / HC, kx = q % HC;
      cplx<T> v[NG];
#pragma unroll
      for (int y = 0; y < NG; ++y) v[y] = s_a1[(z * NG + y) * HC + kx];
      line_dft<T, NG, C, C, false>(v, s_a2 + z * C * HC + kx, HC);
    }
  }
  __syncthreads();
  // z: one column (ky, kx) per lane, all C values of kz, written to the source's spectrum row
  if (work) {
    for (int e = K + lane; e < KP; e += 64) out[e] = {T(0), T(0)};
    for (int col = lane; col < C * HC; col += 64) {
      cplx<T> v[NG];
#pragma unroll
      for (int z = 0; z < NG; ++z) v[z] = s_a2[z * C * HC + col];
      line_dft<T, NG, C, C, false>(v, out + col, C * HC);
    }
  }
}

// Mode chunk of one workgroup of k_cells_accum and the parents it runs side by side: a chunk of
// the Green table of a level (343 offsets x KM modes) is 44 KB of LDS in either precision.
template <typename T>
struct AccumShape {
  static constexpr int KM = sizeof(T) == 4 ? 16 : 8;
  static constexpr int PP = 256 / KM;
};

// One launch per parent level; workgroup (chunk, group): modes [chunk KM, chunk KM + KM) of the
// split parents plist[pbeg + group PP ...], one (parent, mode) per thread. CENTRAL: only the
// sources in the central 4^3 of the block (block coordinates 1..4; the rest of every child's
// zone comes from the transform shared by the parent's children).
template <typename T, int NG, int EXT, bool CENTRAL = false>
__global__ __launch_bounds__(256) void k_cells_accum(CellArgs<T> a, int tlevel, const int* plist,
                                                     int pbeg, int pend) {
  using S = CellShape<NG, EXT>;
  using A = AccumShape<T>;
  constexpr int K = S::KP, KM = A::KM, PP = A::PP;  // the stored rows (zero-padded modes)
  static_assert(K % KM == 0, "mode chunks tile the spectrum");
  // staged offsets: all 7^3 (|d| <= 3), or for the central cubes the 5^3 with |d| <= 2
  constexpr int OW = CENTRAL ? 5 : 7, OR = OW / 2, NOFF = OW * OW * OW;
  __shared__ cplx<T> s_g[NOFF * KM];  // [offset][mode], offset (dx+OR) + OW (dy+OR) + OW^2 (dz+OR)
  __shared__ int s_src[PP * 216];      // source spectrum rows of the group's blocks
  const int tid = threadIdx.x, m = tid % KM, pp = tid / KM;
  const int k0 = blockIdx.x * KM, k = k0 + m;
  const cplx<T>* G = a.gcell + size_t(tlevel - 2) * S::OFFS * K + k0;
  for (int e = tid; e < NOFF * KM; e += 256) {
    const int o = e / KM;
    const int dx = o % OW - OR, dy = (o / OW) % OW - OR, dz = o / (OW * OW) - OR;
    const int o343 = (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3);  // the table's layout
    s_g[e] = G[size_t(o343) * K + e % KM];
  }
  // every group iteration runs in all threads of the workgroup (uniform trip count)
  for (int grp = blockIdx.y; pbeg + grp * PP < pend; grp += gridDim.y) {
    __syncthreads();  // the previous group's slot rows are consumed
    for (int e = tid; e < PP * 216; e += 256) {
      const int q = pbeg + grp * PP + e / 216;
      int v = a.nsources;  // the zero row
      if (q < pend) {
        const int src = a.blocks[size_t(plist[q] - a.first_parent) * 216 + e % 216];
        if (src >= 0) v = src - a.first_cell;
      }
      s_src[e] = v;
    }
    __syncthreads();
    const int idx = pbeg + grp * PP + pp;
    if (idx >= pend) continue;
    const int par = plist[idx];
    const int* row = s_src + pp * 216;
    cplx<T> acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = {T(0), T(0)};
    // two planes at a time in FP32, so that one plane's loads overlap the other's arithmetic
    // (FP64 has no registers to spare for it)
#pragma unroll sizeof(T) == 4 ? 2 : 1
    for (int bz = CENTRAL ? 1 : 0; bz < (CENTRAL ? 5 : 6); ++bz) {
      cplx<T> sp[36];
#pragma unroll
      for (int j = 0; j < 36; ++j) {
        const int jx = j % 6, jy = j / 6;
        if (CENTRAL && (jx < 1 || jx > 4 || jy < 1 || jy > 4)) continue;
        sp[j] = a.sspec[size_t(row[bz * 36 + j]) * K + k];
      }
#pragma unroll
      for (int cz = 0; cz < 2; ++cz) {
        const int dz = bz - 2 - cz;  // in [-3, 3]; in [-2, 2] for the central planes
        const bool zfar = dz < -1 || dz > 1;
        const cplx<T>* gz = s_g + (OW * OW * (dz + OR)) * KM + m;
#pragma unroll
        for (int dy = -3; dy <= 3; ++dy) {
#pragma unroll
          for (int dx = -3; dx <= 3; ++dx) {
            const bool far_xy = dx < -1 || dx > 1 || dy < -1 || dy > 1;
            if (!far_xy && !zfar) continue;  // the 27 offsets of the near zone
            if (CENTRAL && (dx < -2 || dx > 2 || dy < -2 || dy > 2)) continue;  // no central source
            const cplx<T> gv = gz[((dx + OR) + OW * (dy + OR)) * KM];
#pragma unroll
            for (int cy = 0; cy < 2; ++cy) {
#pragma unroll
              for (int cx = 0; cx < 2; ++cx) {
                const int by = dy + 2 + cy, bx = dx + 2 + cx;
                if (by < 0 || by > 5 || bx < 0 || bx > 5) continue;
                if (CENTRAL && (by < 1 || by > 4 || bx < 1 || bx > 4)) continue;
                cplx<T>& o = acc[cx | (cy << 1) | (cz << 2)];
                const cplx<T> sv = sp[by * 6 + bx];
                o.re = fma(gv.re, sv.re, o.re);
                o.re = fma(-gv.im, sv.im, o.re);
                o.im = fma(gv.re, sv.im, o.im);
                o.im = fma(gv.im, sv.re, o.im);
              }
            }
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int t = a.child8[size_t(par) * 8 + c];
      if (t >= 0) a.tspec[size_t(t - a.first_cell) * K + k] = acc[c];
    }
  }
}

// target node t (0 .. NL-1) of an axis sits at cyclic index t - EXT (mod C)
template <int C, int EXT>
__device__ __forceinline__ int cyc(int t) { return t >= EXT ? t - EXT : t - EXT + C; }

// ADD: the target already holds (mean, zero-mean gridlet) from the transform shared by its
// parent's children; this pass adds its own mean and zero-mean part to them (both precisions).
template <typename T, int NG, int EXT, bool ADD = false>
__global__ __launch_bounds__(256) void k_cells_inverse(CellArgs<T> a) {
  using S = CellShape<NG, EXT>;
  constexpr int C = S::C, HC = S::HC, K = S::K, NL = S::NL, M = S::ML;
  constexpr bool split = ADD || sizeof(T) == 4;
  __shared__ cplx<double> tw[C];
  __shared__ cplx<double> s_f[K];              // [kz][ky][kx]
  __shared__ cplx<double> s_b1[NL * C * HC];   // [z][ky][kx], target z
  __shared__ cplx<double> s_b2[NL * NL * HC];  // [z][y][kx]
  __shared__ double s_out[M];
  __shared__ double s_red[4];
  const int t = blockIdx.x, tid = threadIdx.x;
  load_twiddles<double, C>(tw, 1.0);
  const cplx<T>* f = a.tspec + size_t(t) * S::KP;
  for (int e = tid; e < K; e += 256) s_f[e] = {double(f[e].re), double(f[e].im)};
  __syncthreads();
  for (int e = tid; e < NL * C * HC; e += 256) {
    const int col = e % (C * HC), zc = cyc<C, EXT>(e / (C * HC));
    cplx<double> acc = {0.0, 0.0};
    int m = 0;
#pragma unroll
    for (int kz = 0; kz < C; ++kz) {
      acc = cadd(acc, cmul(s_f[kz * C * HC + col], tw[m]));
      m += zc;
      if (m >= C) m -= C;
    }
    s_b1[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < NL * NL * HC; e += 256) {
    const int kx = e % HC, yc = cyc<C, EXT>((e / HC) % NL), z = e / (HC * NL);
    cplx<double> acc = {0.0, 0.0};
    int m = 0;
#pragma unroll
    for (int ky = 0; ky < C; ++ky) {
      acc = cadd(acc, cmul(s_b1[(z * C + ky) * HC + kx], tw[m]));
      m += yc;
      if (m >= C) m -= C;
    }
    s_b2[e] = acc;
  }
  __syncthreads();
  const int g = a.first_cell + t;
  T* out = a.local + size_t(g) * M;
  double part = 0.0;
  for (int e = tid; e < M; e += 256) {
    const int xc = cyc<C, EXT>(e % NL), zy = e / NL;  // zy = z * NL + y
    // real part of the Hermitian sum over kx in (-C/2, C/2]: the kx = 0 and kx = C/2 (Nyquist)
    // terms once, the others twice
    double acc = 0.0;
    int m = 0;
#pragma unroll
    for (int kx = 0; kx < HC; ++kx) {
      const cplx<double> v = s_b2[zy * HC + kx];
      const double re = v.re * tw[m].re - v.im * tw[m].im;
      acc += (kx == 0 || kx == C / 2) ? re : 2.0 * re;
      m += xc;
      if (m >= C) m -= C;
    }
    if constexpr (split) {
      s_out[e] = acc;
      part += acc;
    } else {
      out[e] = T(acc);
    }
  }
  if constexpr (split) {
    part = wave_sum(part);
    if ((tid & 63) == 0) s_red[tid >> 6] = part;
    __syncthreads();
    const double mean = (s_red[0] + s_red[1] + s_red[2] + s_red[3]) * (1.0 / M);
    if constexpr (ADD) {
      for (int e = tid; e < M; e += 256) out[e] = T(double(out[e]) + (s_out[e] - mean));
      if (tid == 0) a.m2l_mean[g] += mean;
    } else {
      for (int e = tid; e < M; e += 256) out[e] = T(s_out[e] - mean);
      if (tid == 0) a.m2l_mean[g] = mean;
    }
  }
}

// SHARED: the route with the transform shared by siblings (the central cubes here, the outer
// cubes by the per-parent kernel before the inverse adds to its result)
template <typename T, int NG, int EXT, bool SHARED = false>
static void cells_t(Plan& p, hipStream_t s) {
  using S = CellShape<NG, EXT>;
  p.m2l_split = SHARED || sizeof(T) == 4;
  p.m2l_mean_ff = false;  // this route's means are doubles
  if (p.nlevels <= 2) return;
  CellArgs<T> a;
  a.first_cell = p.level_off[2];
  const int ntargets = int(p.ncells) - a.first_cell;
  if (ntargets <= 0) return;
  a.nsources = ntargets + int(p.nvirt);
  a.first_parent = p.blocks_first;
  a.nlevels = p.nlevels;
  a.level_off = p.dlev.as<int>() + kLevOff;
  a.child8 = p.child8.as<int>();
  a.blocks = p.blocks.as<int>();
  a.gridlet = p.gridlet.as<T>();
  a.local = p.local.as<T>();
  a.gcell = p.tab.gcell.as<cplx<T>>();
  a.sspec = p.cell_src.as<cplx<T>>();
  a.tspec = p.cell_tgt.as<cplx<T>>();
  a.m2l_mean = p.m2l_mean.as<double>();
  if (p.tab.gcell_levels < p.nlevels - 2) fail(HPM_ERR_DEVICE, "cell Green tables missing");
  if (p.cell_src.bytes < size_t(a.nsources + 1) * S::KP * sizeof(cplx<T>) ||
      p.cell_tgt.bytes < size_t(ntargets) * S::KP * sizeof(cplx<T>) ||
      p.local.bytes < size_t(p.ncells) * S::ML * sizeof(T))
    fail(HPM_ERR_DEVICE, "cell spectra buffers too small");
  k_cells_forward<T, NG, EXT><<<(a.nsources + kFwdSources) / kFwdSources, kFwdThreads, 0, s>>>(a);
  HPM_LAUNCH_CHECK();
  using A = AccumShape<T>;
  for (int lp = 1; lp + 1 < p.nlevels; ++lp) {
    const int pbeg = p.cell_pbeg[lp], pend = p.cell_pbeg[lp + 1];
    if (pend <= pbeg) continue;
    const int groups = std::min((pend - pbeg + A::PP - 1) / A::PP, 65535);
    k_cells_accum<T, NG, EXT, SHARED><<<dim3(S::KP / A::KM, groups), 256, 0, s>>>(
        a, lp + 1, p.cell_plist.as<int>(), pbeg, pend);
    HPM_LAUNCH_CHECK();
  }
  if constexpr (SHARED) launch_m2l_parents(p, s);
  k_cells_inverse<T, NG, EXT, SHARED><<<ntargets, 256, 0, s>>>(a);
  HPM_LAUNCH_CHECK();
}

size_t cell_modes(int ng, int ext) {
  const size_t c = size_t(2 * ng + 2 * ext), k = c * c * (c / 2 + 1);
  return (k + 15) / 16 * 16;
}

// ---- list of split parents (cells of levels 1 .. L-2 with children), by level ----------------
// The list itself is written by the tree build; the start of each parent level in it is in the
// mailbox.
void read_cell_parents(Plan& p) {
  for (int l = 0; l <= kMaxLevelsHost; ++l) p.cell_pbeg[l] = 0;
  if (p.nlevels <= 2 || p.level_off[p.nlevels - 1] <= p.level_off[1]) return;
  for (int l = 1; l <= p.nlevels - 1; ++l) p.cell_pbeg[l] = p.hbox[Plan::kBoxCellLevels + l];
}

template <typename T>
static void cells_dispatch(Plan& p, hipStream_t s) {
  switch (p.ng * 2 + p.ext) {
    case 4: cells_t<T, 2, 0>(p, s); break;
    case 5: cells_t<T, 2, 1>(p, s); break;
    case 6: cells_t<T, 3, 0>(p, s); break;
    case 7: cells_t<T, 3, 1>(p, s); break;
    case 8: cells_t<T, 4, 0>(p, s); break;
    case 9: cells_t<T, 4, 1>(p, s); break;
    case 12: cells_t<T, 6, 0>(p, s); break;
    case 13: cells_t<T, 6, 1>(p, s); break;
    case 16: cells_t<T, 8, 0>(p, s); break;
    default: fail(HPM_ERR_UNSUPPORTED, "no cell-by-cell kernels for this gridlet");
  }
}

void launch_m2l_cells(Plan& p, hipStream_t s) {
  if (p.prec == HPM_F32) cells_dispatch<float>(p, s);
  else cells_dispatch<double>(p, s);
}

template <typename T>
static void shared_dispatch(Plan& p, hipStream_t s) {
  if (p.ext) fail(HPM_ERR_UNSUPPORTED, "the shared-transform route has no extended gridlet");
  switch (p.ng) {
    case 2: cells_t<T, 2, 0, true>(p, s); break;
    case 3: cells_t<T, 3, 0, true>(p, s); break;
    case 4: cells_t<T, 4, 0, true>(p, s); break;
    case 6: cells_t<T, 6, 0, true>(p, s); break;
    default: fail(HPM_ERR_UNSUPPORTED, "no shared-transform kernels for this gridlet");
  }
}

void launch_m2l_shared(Plan& p, hipStream_t s) {
  if (p.prec == HPM_F32) shared_dispatch<float>(p, s);
  else shared_dispatch<double>(p, s);
}

}  // namespace hpm
