// Source-to-target (M2L) by one zero-padded FFT per target (Sec. 2.1, Eq. 1).
//
// For a target T at level l >= 2 with parent P and octant c, the effective masses of the 216
// level-l cubes of the 6^3 block around P (block cube b at lattice offset b N_g), minus the 27
// cubes touching T, are placed on an n^3 grid, n = 8 N_g (the padding that is exact for the
// target, Sec. 2.1); the grid is transformed, multiplied by the transform of the exact lattice
// Green function of level l, transformed back, and the N_g^3 values at [(2 + c) N_g, (3 + c) N_g)
// per axis are the target's gridlet potentials.
//
// One workgroup per target. The forward transform is pruned where the input is known to be
// zero (the grid is nonzero only in [0, 6 N_g)^3) and the inverse where the output is not
// needed (only N_g values per axis), which is the paper's output-pruning remark (Sec. 2.1)
// applied per pass; every transform is an in-register line FFT:
//   x : rows (y, z) < 6 N_g, two real rows per complex FFT, half spectrum kx <= n/2 kept
//   y : columns (kx, z < 6 N_g)
//   z : columns (kx, ky), multiplied by the Green transform (real and even, octant table),
//       inverse z FFT, the N_g target z values kept
//   y^-1 : columns (kx, z' < N_g), the N_g target y values kept
//   x^-1 : rows (y', z'), Hermitian half spectrum -> the N_g target x values
// The line buffer ("stage", layout [z < 6N_g][y < n][kx <= n/2] complex) lives in LDS; this
// kernel serves N_g <= 3, the z-slab kernel below the larger orders. Cubes of the interaction zone that are
// not cells of the tree but lie inside a coarser leaf ("virtual" cubes) have their effective
// masses fitted once per solve, beside the leaves'; they are found here by their cube id.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dev_common.h"
#include "fft.h"
#include "hpm_internal.h"

namespace hpm {

template <typename T, int NG>
struct M2LShape {
  static constexpr int n = 8 * NG;
  static constexpr int H = n / 2 + 1;
  static constexpr int W = 6 * NG;
  static constexpr int M = NG * NG * NG;
  static constexpr size_t elems = size_t(W) * n * H;
  static constexpr size_t bytes = elems * sizeof(cplx<T>);
  static constexpr bool lds = bytes <= 112 * 1024;
};

template <typename T>
struct M2LArgs {
  int first_target;
  int ntargets;
  int nlevels;
  int depth;
  const int* level_off;
  const int* coord;
  const int* parent;
  const int* blocks;  // [parent][216] source gridlet ids of each parent's block (or -1)
  int first_parent;   // cell id of the table's first row
  const T* gridlet;
  T* local;
  double* m2l_mean;  // z-slab kernel: mean of each target's result (the gridlet part is zero-mean)
  const float4* twff;  // FP32 plans: e^{+2 pi i m / n} as {cos hi, sin hi, cos lo, sin lo}
  const T* ghat;
  const T* gxy;
  double lo0, lo1, lo2, size;
  // per-parent kernel: the split parents (cell ids) and every cell's 8 children (or -1)
  const int* plist;
  int nparents;
  const int* child8;
};

constexpr int fold_k(int k, int n) { return k <= n / 2 ? k : n - k; }

struct TargetGeom {
  int g, l, tx, ty, tz, cx, cy, cz, par;
  double L;
};

__device__ __forceinline__ TargetGeom target_geom(int g, const int* s_off, int nlevels,
                                                  const int* coord, const int* parent, double size) {
  TargetGeom t;
  t.g = g;
  t.l = level_of(g, s_off, nlevels);
  const int pc = coord[g];
  t.tx = coord_x(pc);
  t.ty = coord_y(pc);
  t.tz = coord_z(pc);
  t.cx = t.tx & 1;
  t.cy = t.ty & 1;
  t.cz = t.tz & 1;
  t.par = parent[g];
  t.L = size / double(1 << t.l);
  return t;
}

// Source of block cube "slot" (< 216) of target t: its gridlet id (a real cell, or ncells + v
// for a virtual cube), or -1 for the 27 cubes around the target and for empty positions.
template <typename T>
__device__ __forceinline__ int resolve_slot(const M2LArgs<T>& a, const TargetGeom& t, int slot) {
  const int bx = slot % 6, by = (slot / 6) % 6, bz = slot / 36;
  const bool near = abs(bx - 2 - t.cx) <= 1 && abs(by - 2 - t.cy) <= 1 && abs(bz - 2 - t.cz) <= 1;
  return near ? -1 : a.blocks[size_t(t.par - a.first_parent) * 216 + slot];
}

// x pass of the two source rows (y0, zr) and (y0 + 1, zr) of the block grid (y0 even): the
// gridlet rows of the six cubes along x are gathered into one complex line (first row real,
// second imaginary), transformed, and split into the half spectra A and B of the two real rows.
template <typename T, int NG>
__device__ __forceinline__ void xpass_rows(const M2LArgs<T>& a, int y0, int zr, const int* s_src,
                                           cplx<T> (&A)[4 * NG + 1], cplx<T> (&B)[4 * NG + 1]) {
  constexpr int n = 8 * NG, M = NG * NG * NG, H = 4 * NG + 1;
  cplx<T> line[n];
#pragma unroll
  for (int k = 0; k < n; ++k) line[k] = {T(0), T(0)};
  const int bz = zr / NG, kz = zr % NG;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int yr = y0 + half;
    const int by = yr / NG, jy = yr % NG;
#pragma unroll
    for (int bx = 0; bx < 6; ++bx) {
      const int src = s_src[bx + 6 * (by + 6 * bz)];
      if (src >= 0) {
        const T* gsrc = a.gridlet + size_t(src) * M + (kz * NG + jy) * NG;
#pragma unroll
        for (int i = 0; i < NG; ++i) {
          if (half == 0) line[bx * NG + i].re = gsrc[i];
          else line[bx * NG + i].im = gsrc[i];
        }
      }
    }
  }
  cplx<T> zf[n];
  fft<n, -1>(line, zf);
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const cplx<T> z1 = zf[k], z2 = zf[(n - k) % n];
    A[k] = {T(0.5) * (z1.re + z2.re), T(0.5) * (z1.im - z2.im)};
    B[k] = {T(0.5) * (z1.im + z2.im), T(0.5) * (z2.re - z1.re)};
  }
}

// x pass of one source row (y, zr) of the block grid: the gridlet rows of the six cubes along x
// (6 N_g values, zero beyond) as a real line of length n = 8 N_g, whose half spectrum
// X[0..n/2] comes from one n/2-point complex FFT of the packed even/odd samples:
//   Z = FFT(x[2j] + i x[2j+1]),  E_k = (Z_k + conj Z_{n/2-k}) / 2,  O_k = (Z_k - conj Z_{n/2-k}) / 2i,
//   X_k = E_k + e^{-2 pi i k / n} O_k.
template <typename T, int NG>
__device__ __forceinline__ void xpass_row(const M2LArgs<T>& a, int yr, int zr, const int* s_src,
                                          cplx<T> (&X)[4 * NG + 1]) {
  constexpr int n = 8 * NG, h = n / 2, M = NG * NG * NG;
  cplx<T> z[h];
#pragma unroll
  for (int j = 0; j < h; ++j) z[j] = {T(0), T(0)};
  const int bz = zr / NG, kz = zr % NG, by = yr / NG, jy = yr % NG;
#pragma unroll
  for (int bx = 0; bx < 6; ++bx) {
    const int src = s_src[bx + 6 * (by + 6 * bz)];
    if (src >= 0) {
      const T* gsrc = a.gridlet + size_t(src) * M + (kz * NG + jy) * NG;
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        const int xx = bx * NG + i;  // compile-time: even samples real, odd imaginary
        if (xx % 2 == 0) z[xx / 2].re = gsrc[i];
        else z[xx / 2].im = gsrc[i];
      }
    }
  }
  cplx<T> Z[h];
  fft<h, -1>(z, Z);
  static_for<0, h + 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const cplx<T> zk = Z[k % h], zc = Z[(h - k) % h];
    const cplx<T> e = {T(0.5) * (zk.re + zc.re), T(0.5) * (zk.im - zc.im)};
    const cplx<T> o = {T(0.5) * (zk.im + zc.im), T(0.5) * (zc.re - zk.re)};
    const cplx<T> wo = twiddle<k, n, -1>(o);
    X[k] = {e.re + wo.re, e.im + wo.im};
  });
}

// The same half spectrum split over two threads by the parity Q of k (decimation in frequency of
// the n/2-point transform: its even outputs are the n/4-point transform of z_j + z_{j+n/4}, its odd
// ones that of (z_j - z_{j+n/4}) e^{-2 pi i j / (n/2)}; X_k needs Z_k and Z_{n/2-k}, both of parity
// Q). The thread writes X_k for k = Q, Q + 2, ... <= n/2 into row[k].
template <typename T, int NG, int Q>
__device__ __forceinline__ void xpass_row_half(const M2LArgs<T>& a, int yr, int zr, const int* s_src,
                                               cplx<T>* row) {
  constexpr int n = 8 * NG, h = n / 2, hh = h / 2, M = NG * NG * NG, W = 6 * NG;
  T x[n];
#pragma unroll
  for (int j = 0; j < n; ++j) x[j] = T(0);
  const int bz = zr / NG, kz = zr % NG, by = yr / NG, jy = yr % NG;
#pragma unroll
  for (int bx = 0; bx < 6; ++bx) {
    const int src = s_src[bx + 6 * (by + 6 * bz)];
    if (src >= 0) {
      const T* gsrc = a.gridlet + size_t(src) * M + (kz * NG + jy) * NG;
#pragma unroll
      for (int i = 0; i < NG; ++i) x[bx * NG + i] = gsrc[i];
    }
  }
  cplx<T> u[hh], Zq[hh];
  static_for<0, hh>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    const cplx<T> z0 = {x[2 * j], x[2 * j + 1]};
    const cplx<T> z1 = (2 * j + h < W) ? cplx<T>{x[2 * j + h], x[2 * j + h + 1]} : cplx<T>{T(0), T(0)};
    if constexpr (Q == 0) u[j] = cadd(z0, z1);
    else u[j] = twiddle<j, h, -1>(csub(z0, z1));
  });
  fft<hh, -1>(u, Zq);  // Zq[kk] = Z[2 kk + Q]
  static_for<0, hh + 1>([&](auto kc) {
    constexpr int k = 2 * decltype(kc)::value + Q;
    if constexpr (k <= h) {
      const cplx<T> zk = Zq[(k % h) / 2], zc = Zq[((h - k) % h) / 2];
      const cplx<T> e = {T(0.5) * (zk.re + zc.re), T(0.5) * (zk.im - zc.im)};
      const cplx<T> o = {T(0.5) * (zk.im + zc.im), T(0.5) * (zc.re - zk.re)};
      const cplx<T> wo = twiddle<k, n, -1>(o);
      row[k] = {e.re + wo.re, e.im + wo.im};
    }
  });
}

template <typename T, int NG>
__global__ __launch_bounds__(256) void k_m2l(M2LArgs<T> a) {
  using S = M2LShape<T, NG>;
  constexpr int n = S::n, H = S::H, W = S::W, M = S::M;
  __shared__ int s_src[216];
  __shared__ int s_off[kMaxLevels + 1];
  static_assert(S::lds, "the whole-grid kernel keeps its stage in LDS");
  __shared__ cplx<T> stage[S::elems];
  const int tid = threadIdx.x;
  if (tid <= kMaxLevels) s_off[tid] = a.level_off[tid];

  // The 8 XCDs take contiguous chunks of the Morton-ordered targets (neighbouring targets
  // share most of their interaction zones, so their gridlets stay in the XCD's L2).
  const int xcd = blockIdx.x & 7, per = gridDim.x >> 3, j = blockIdx.x >> 3;
  const int t_begin = int((int64_t(a.ntargets) * xcd) / 8);
  const int t_end = int((int64_t(a.ntargets) * (xcd + 1)) / 8);

  for (int ti = t_begin + j; ti < t_end; ti += per) {
    __syncthreads();
    const TargetGeom t = target_geom(a.first_target + ti, s_off, a.nlevels, a.coord, a.parent, a.size);
    const int g = t.g, l = t.l, cx = t.cx, cy = t.cy, cz = t.cz;
    if (tid < 216) s_src[tid] = resolve_slot(a, t, tid);
    __syncthreads();

    // ---- x: gather two rows, real-to-complex --------------------------------------------------
    for (int w = tid; w < W * W / 2; w += blockDim.x) {
      const int r0 = 2 * w;
      const int y0 = r0 % W, zr = r0 / W;  // rows (y0, zr) and (y0 + 1, zr)
      cplx<T> A[H], B[H];
      xpass_rows<T, NG>(a, y0, zr, s_src, A, B);
      cplx<T>* row0 = stage + (size_t(zr) * n + y0) * H;
      cplx<T>* row1 = row0 + H;
#pragma unroll
      for (int k = 0; k < H; ++k) {
        row0[k] = A[k];
        row1[k] = B[k];
      }
    }
    __syncthreads();

    // ---- y: columns (kx, z < W) ---------------------------------------------------------------
    for (int w = tid; w < H * W; w += blockDim.x) {
      const int kx = w % H, zr = w / H;
      cplx<T>* col = stage + size_t(zr) * n * H + kx;
      cplx<T> in[n], out[n];
#pragma unroll
      for (int y = 0; y < n; ++y) in[y] = (y < W) ? col[size_t(y) * H] : cplx<T>{T(0), T(0)};
      fft<n, -1>(in, out);
#pragma unroll
      for (int y = 0; y < n; ++y) col[size_t(y) * H] = out[y];
    }
    __syncthreads();

    // ---- z: columns (kx, ky), Green multiply, inverse z, keep the target's N_g z values --------
    const T* gl = a.ghat + size_t(l - 2) * H * H * H;
    for (int w = tid; w < H * n; w += blockDim.x) {
      const int kx = w % H, ky = w / H;
      const int kyf = ky <= n / 2 ? ky : n - ky;
      cplx<T>* col = stage + size_t(ky) * H + kx;
      constexpr size_t zs = size_t(n) * H;
      cplx<T> in[n], out[n];
#pragma unroll
      for (int z = 0; z < n; ++z) in[z] = (z < W) ? col[z * zs] : cplx<T>{T(0), T(0)};
      fft<n, -1>(in, out);
#pragma unroll
      for (int kz = 0; kz < n; ++kz) {
        const T gv = gl[(size_t(fold_k(kz, n)) * H + kyf) * H + kx];
        out[kz] = cscale(out[kz], gv);
      }
      fft<n, +1>(out, in);
#pragma unroll
      for (int zz = 0; zz < NG; ++zz) col[zz * zs] = cz ? in[3 * NG + zz] : in[2 * NG + zz];
    }
    __syncthreads();

    // ---- y^-1: columns (kx, z' < N_g), keep the target's N_g y values -------------------------
    for (int w = tid; w < H * NG; w += blockDim.x) {
      const int kx = w % H, zz = w / H;
      cplx<T>* col = stage + size_t(zz) * n * H + kx;
      cplx<T> in[n], out[n];
#pragma unroll
      for (int y = 0; y < n; ++y) in[y] = col[size_t(y) * H];
      fft<n, +1>(in, out);
#pragma unroll
      for (int yy = 0; yy < NG; ++yy) col[size_t(yy) * H] = cy ? out[3 * NG + yy] : out[2 * NG + yy];
    }
    __syncthreads();

    // ---- x^-1: two Hermitian rows per complex FFT, keep the target's N_g x values -------------
    for (int w = tid; w < (NG * NG + 1) / 2; w += blockDim.x) {
      const int r0 = 2 * w, r1 = 2 * w + 1;
      const bool has1 = r1 < NG * NG;
      const cplx<T>* A = stage + (size_t(r0 / NG) * n + (r0 % NG)) * H;
      const cplx<T>* B = stage + (size_t(r1 / NG) * n + (r1 % NG)) * H;
      cplx<T> zf[n], zo[n];
#pragma unroll
      for (int k = 0; k < H; ++k) {
        cplx<T> av = A[k], bv = has1 ? B[k] : cplx<T>{T(0), T(0)};
        if (k == 0 || k == n / 2) {
          av.im = T(0);
          bv.im = T(0);
        }
        zf[k] = {av.re - bv.im, av.im + bv.re};
        if (k > 0 && k < n / 2) zf[n - k] = {av.re + bv.im, bv.re - av.im};
      }
      fft<n, +1>(zf, zo);
      T* out0 = a.local + size_t(g) * M + r0 * NG;
#pragma unroll
      for (int xx = 0; xx < NG; ++xx) out0[xx] = cx ? zo[3 * NG + xx].re : zo[2 * NG + xx].re;
      if (has1) {
        T* out1 = a.local + size_t(g) * M + r1 * NG;
#pragma unroll
        for (int xx = 0; xx < NG; ++xx) out1[xx] = cx ? zo[3 * NG + xx].im : zo[2 * NG + xx].im;
      }
    }
  }
}


// ---------------------------------------------------------------------------------------------
// z-slab variant: the same convolution, streamed over the source z rows.
//
// The source grid is taken ZB z-rows (one "slab") at a time. Each slab is transformed along x
// (two real rows per complex FFT, half spectrum kx <= n/2) and along y (all n values of ky) in
// LDS. Along z the convolution is written out in real space: for the N_g target z values Z and
// a source row z, the kernel is the Green function transformed along x and y only, at the
// offset |Z - z| < 4 N_g (no wrap-around), so
//     P(Z, ky, kx) = sum_z Gxy(|Z - z|, ky, kx) S(z, ky, kx)
// accumulates in registers, one (ky, kx) entry per thread slot, slab by slab. Once every slab
// is in, the N_g planes P(Z) go through the inverse y transform (N_g target y values kept) and
// the Hermitian inverse x transform (N_g target x values kept). Nothing but the source gridlets
// and the N_g^3 outputs crosses the memory hierarchy, and the forward z transform, the Green
// multiply and the inverse z transform of the full-grid kernel are replaced by N_g x 6 N_g
// real multiply-adds per (ky, kx) entry.
// ---------------------------------------------------------------------------------------------
constexpr int kSlabThreads = 256;      // threads per workgroup
constexpr int kSlabLayers = 1;         // block layers (N_g source z rows each) per slab
constexpr bool kSlabGreenLds = false;  // Green table of the level in LDS (else read through L2)
constexpr int kSlabPerCU = 2;          // resident workgroups per CU

// EXT = 1: extended target gridlets (Sec. 2.5), NL = N_g + 2 nodes per axis, the target window
// [(2 + c) N_g - 1, (3 + c) N_g + 1) per axis.
template <typename T, int NG, int EXT = 0>
struct SlabShape {
  static constexpr int n = 8 * NG, H = n / 2 + 1, W = 6 * NG, M = NG * NG * NG;
  static constexpr int NL = NG + 2 * EXT, ML = NL * NL * NL;  // target gridlet
  static constexpr int NT = kSlabThreads;
  // At N_g = 8 the inverse y transform is a pruned direct sum in double (FP32 rounding of the
  // inverse transforms would dominate the gradient of a degree-7 interpolant), and its output
  // buffer in double leaves room for half a block layer per slab. FP64 at N_g = 8 also cannot
  // hold the accumulators of all N_g target planes (288 registers per thread): it streams two
  // source rows per slab, forms the target planes in two passes of N_g / 2, and splits each x
  // line over two threads and each forward y line over four.
  static constexpr bool wide = NG >= 8;
  static constexpr bool narrow = wide && sizeof(T) == 8;
  static constexpr int ZB = wide ? (narrow ? 2 : NG / 2) : kSlabLayers * NG;  // source rows per slab
  static constexpr int ZW = narrow ? NG / 2 : NL;           // target z planes per pass
  static constexpr int YS = narrow ? 4 : 1;                 // threads per forward y line
  static constexpr int XS = narrow ? 2 : 1;                 // threads per x line
  static constexpr int ZG = ZB < ZW ? ZB : ZW;              // planes per inverse-y group
  using RedT = typename std::conditional<wide, double, T>::type;  // inverse-y output
  static constexpr int D = 4 * NG + 1;      // z offsets |Z - z| <= 4 N_g (table rows)
  static constexpr int ENT = n * H;         // (ky, kx) entries of a plane
  static constexpr int PER = (ENT + NT - 1) / NT;
  static constexpr int NJ = ZW + ZB - 1;    // distinct offsets Z - z within one slab and pass
  static constexpr size_t slab_bytes = size_t(ZB) * n * H * sizeof(cplx<T>);
  static constexpr size_t green_bytes = size_t(D) * H * H * sizeof(T);
  static constexpr size_t red_bytes = size_t(NL) * NL * H * sizeof(cplx<RedT>) + size_t(ML) * 8 +
                                      size_t(n) * sizeof(cplx<double>) + 2048;
  static constexpr bool green_lds =
      kSlabGreenLds && slab_bytes + red_bytes + green_bytes <= 160 * 1024;
  static constexpr bool fits = slab_bytes + red_bytes <= 160 * 1024;
};

// The slab loop of the z-slab scheme: every source z row of the 6 N_g block (the cubes of s_src)
// through the x and y transforms in LDS and into the real-space z sum (pr, pi) at the ZW target
// z values Zt .. Zt + ZW - 1. Called by all threads of the workgroup; the accumulators are
// per thread, entry e = tid + NT r. tw holds e^{+2 pi i m / n}, m < n.
template <typename T, int NG, int EXT = 0>
__device__ __forceinline__ void slab_sum(const M2LArgs<T>& a, const int* s_src, cplx<T>* slab,
                                         const T* gtab, int Zt, const cplx<double>* tw,
                                         T (&pr)[SlabShape<T, NG, EXT>::PER][SlabShape<T, NG, EXT>::ZW],
                                         T (&pi)[SlabShape<T, NG, EXT>::PER][SlabShape<T, NG, EXT>::ZW]) {
  using S = SlabShape<T, NG, EXT>;
  constexpr int n = S::n, H = S::H, W = S::W, NT = S::NT, ZB = S::ZB, ZW = S::ZW, YS = S::YS,
                PER = S::PER, NJ = S::NJ, ENT = S::ENT;
  const int tid = threadIdx.x;
#pragma unroll
  for (int r = 0; r < PER; ++r)
#pragma unroll
    for (int zz = 0; zz < ZW; ++zz) pr[r][zz] = pi[r][zz] = T(0);

  for (int z0 = 0; z0 < W; z0 += ZB) {
    if constexpr (S::XS == 1) {
      // x: rows (zb, y) of the slab, y fastest, one real row per thread
      for (int w = tid; w < ZB * W; w += NT) {
        const int zb = w / W, yr = w % W;
        cplx<T> X[H];
        xpass_row<T, NG>(a, yr, z0 + zb, s_src, X);
        cplx<T>* row = slab + (size_t(zb) * n + yr) * H;
#pragma unroll
        for (int k = 0; k < H; ++k) row[k] = X[k];
      }
    } else {
      // x: two threads per row, one per parity of the output frequency
      for (int w = tid; w < ZB * W * 2; w += NT) {
        const int q = w & 1, r = w >> 1;
        const int zb = r / W, yr = r % W;
        cplx<T>* row = slab + (size_t(zb) * n + yr) * H;
        if (q == 0) xpass_row_half<T, NG, 0>(a, yr, z0 + zb, s_src, row);
        else xpass_row_half<T, NG, 1>(a, yr, z0 + zb, s_src, row);
      }
    }
    __syncthreads();
    if constexpr (YS == 1) {
      // y: columns (zb, kx); rows y >= 6 N_g are zero
      for (int w = tid; w < ZB * H; w += NT) {
        const int kx = w % H, zb = w / H;
        cplx<T>* col = slab + size_t(zb) * n * H + kx;
        cplx<T> in[n], out[n];
#pragma unroll
        for (int y = 0; y < n; ++y) in[y] = (y < W) ? col[size_t(y) * H] : cplx<T>{T(0), T(0)};
        fft<n, -1>(in, out);
#pragma unroll
        for (int y = 0; y < n; ++y) col[size_t(y) * H] = out[y];
      }
    } else {
      // y split over YS threads per column (decimation in frequency): thread q transforms
      //   u_j = e^{-2 pi i q j / n} sum_r x_{j + r m} e^{-2 pi i q r / YS},  j < m = n / YS,
      // whose m-point transform is the column's outputs ky = YS k + q. All threads read their
      // inputs before any output is written back in place.
      static_assert(YS == 4, "forward y split");
      constexpr int m = n / YS, TASKS = ZB * H * YS;
      for (int w0 = 0; w0 < TASKS; w0 += NT) {
        const int w = w0 + tid;
        const bool live = w < TASKS;
        const int q = w % YS, c = w / YS;
        const int kx = c % H, zb = c / H;
        cplx<T>* col = slab + size_t(zb) * n * H + kx;
        cplx<T> u[m], out[m];
        if (live) {
#pragma unroll
          for (int j = 0; j < m; ++j) {
            cplx<T> acc = {T(0), T(0)};
#pragma unroll
            for (int r = 0; r < YS; ++r) {
              if (j + r * m < W) {
                const cplx<T> v = col[size_t(j + r * m) * H];
                // times (-i)^(q r)
                switch ((q * r) & 3) {
                  case 0: acc = cadd(acc, v); break;
                  case 1: acc = cadd(acc, cplx<T>{v.im, -v.re}); break;
                  case 2: acc = csub(acc, v); break;
                  default: acc = cadd(acc, cplx<T>{-v.im, v.re}); break;
                }
              }
            }
            const cplx<double> t = tw[(q * j) % n];
            u[j] = cmul(acc, cplx<T>{T(t.re), T(-t.im)});
          }
          fft<m, -1>(u, out);
        }
        __syncthreads();
        if (live) {
#pragma unroll
          for (int k = 0; k < m; ++k) col[size_t(YS * k + q) * H] = out[k];
        }
        __syncthreads();
      }
    }
    __syncthreads();
    // z in real space: P(Z) += sum_zb Gxy(|Zt + Z - z0 - zb|) S(zb) for this slab, the slab's
    // terms chained with FMAs before they join the running sum
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + NT * r;
      if (e < ENT) {
        const int ky = e / H, kx = e % H;
        const int kyf = ky <= n / 2 ? ky : n - ky;
        T g[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int d = Zt - z0 + j - (ZB - 1);
          g[j] = gtab[(size_t(d < 0 ? -d : d) * H + kyf) * H + kx];
        }
        cplx<T> sv[ZB];
#pragma unroll
        for (int zb = 0; zb < ZB; ++zb) sv[zb] = slab[(size_t(zb) * n + ky) * H + kx];
#pragma unroll
        for (int zz = 0; zz < ZW; ++zz) {
          T ar = g[zz + ZB - 1] * sv[0].re, ai = g[zz + ZB - 1] * sv[0].im;
#pragma unroll
          for (int zb = 1; zb < ZB; ++zb) {
            const T gv = g[zz - zb + ZB - 1];
            ar = fma(gv, sv[zb].re, ar);
            ai = fma(gv, sv[zb].im, ai);
          }
          pr[r][zz] += ar;
          pi[r][zz] += ai;
        }
      }
    }
    __syncthreads();
  }
}

// STRICT (FP32 plans, N_g = 4 and 6): the inverse x sums and the mean in float-float arithmetic
// against float-float twiddles from the tables, the mean stored as a float pair; no FP64
// arithmetic in the kernel.
template <typename T, int NG, int EXT, bool STRICT = false>
__global__ __launch_bounds__(kSlabThreads) void k_m2l_slab(M2LArgs<T> a) {
  using S = SlabShape<T, NG, EXT>;
  static_assert(!STRICT || (sizeof(T) == 4 && !S::wide), "float-float inverse: FP32, N_g <= 6");
  constexpr int n = S::n, H = S::H, NT = S::NT, D = S::D, PER = S::PER, ENT = S::ENT,
                ZW = S::ZW, ZG = S::ZG, NL = S::NL, ML = S::ML;
  static_assert(S::fits, "slab buffers exceed the LDS budget");
  static_assert(S::W % S::ZB == 0 && S::W % 2 == 0 && NL % ZW == 0, "slab shape");
  __shared__ int s_src[216];
  __shared__ int s_off[kMaxLevels + 1];
  __shared__ __align__(16) cplx<T> slab[S::ZB * n * H];  // [zb][ky (y before the y pass)][kx]
  __shared__ cplx<typename S::RedT> red[NL * NL * H];    // after y^-1: [Z][Y][kx]
  __shared__ double s_out[ML];
  __shared__ double s_red[NT / 64];
  __shared__ cplx<double> s_tw[n];  // e^{+2 pi i m / n}
  __shared__ T s_green[S::green_lds ? D * H * H : 1];  // [d][ky folded][kx]
  __shared__ float4 s_twf[STRICT ? n : 1];
  const int tid = threadIdx.x;
  // Waves of this kernel win issue arbitration over the near-zone kernel running beside it on
  // the second stream (measured: 1% off the solve, and off this kernel alone as well).
  __builtin_amdgcn_s_setprio(2);
  if (tid <= kMaxLevels) s_off[tid] = a.level_off[tid];
  for (int m = tid; m < n; m += NT) {
    if constexpr (STRICT) {
      s_twf[m] = a.twff[m];
    } else {
      double sv, cv;
      sincospi(2.0 * m / n, &sv, &cv);
      s_tw[m] = {cv, sv};
    }
  }
  int green_level = -1;

  const int xcd = blockIdx.x & 7, per = gridDim.x >> 3, jb = blockIdx.x >> 3;
  const int t_begin = int((int64_t(a.ntargets) * xcd) / 8);
  const int t_end = int((int64_t(a.ntargets) * (xcd + 1)) / 8);

  for (int ti = t_begin + jb; ti < t_end; ti += per) {
    __syncthreads();
    const TargetGeom t = target_geom(a.first_target + ti, s_off, a.nlevels, a.coord, a.parent, a.size);
    if (tid < 216) s_src[tid] = resolve_slot(a, t, tid);
    const T* gtab_g = a.gxy + size_t(t.l - 2) * D * H * H;
    if constexpr (S::green_lds) {
      if (t.l != green_level) {  // block-uniform: every thread sees the same target
        for (int e = tid; e < D * H * H; e += NT) s_green[e] = gtab_g[e];
        green_level = t.l;
      }
    }
    __syncthreads();
    const T* gtab = S::green_lds ? s_green : gtab_g;
    const int Zt = (2 + t.cz) * NG - EXT;

    // The target z planes in passes of ZW (all N_g at once unless the accumulators would not
    // fit), each pass's planes through the slab buffer ZG at a time for the inverse y transform.
    // The inverse y transform runs in the plan's precision (the N_g target values of each column
    // kept) and the inverse x transform in double precision as direct sums against a double
    // twiddle table: the last rounding then happens at the magnitude of the potential's variation
    // across the target, not at that of the interaction zone's large smooth potential.
    for (int zp = 0; zp < NL; zp += ZW) {
      T pr[PER][ZW], pi[PER][ZW];
      slab_sum<T, NG, EXT>(a, s_src, slab, gtab, Zt + zp, s_tw, pr, pi);
#pragma unroll
      for (int z0 = 0; z0 < ZW; z0 += ZG) {
        const int zg = ZW - z0 < ZG ? ZW - z0 : ZG;  // planes in this group
#pragma unroll
        for (int r = 0; r < PER; ++r) {
          const int e = tid + NT * r;
          if (e < ENT) {
#pragma unroll
            for (int zz = 0; zz < ZG; ++zz)
              if (z0 + zz < ZW) slab[size_t(zz) * ENT + e] = {pr[r][z0 + zz], pi[r][z0 + zz]};
          }
        }
        __syncthreads();
        // y^-1: red[Z][yy][kx] = sum_ky P(Z, ky, kx) e^{+2 pi i ky Y / n},
        // Y = (2 + c_y) N_g - EXT + yy
        if constexpr (!S::wide) {
          for (int w = tid; w < zg * H; w += NT) {
            const int kx = w % H, zz = w / H;
            const cplx<T>* col = slab + size_t(zz) * ENT + kx;
            cplx<T> in[n], out[n];
#pragma unroll
            for (int y = 0; y < n; ++y) in[y] = col[size_t(y) * H];
            fft<n, +1>(in, out);
#pragma unroll
            for (int yy = 0; yy < NL; ++yy) {
              const cplx<T> o0 = out[2 * NG - EXT + yy], o1 = out[3 * NG - EXT + yy];
              red[(size_t(zp + z0 + zz) * NL + yy) * H + kx] = {t.cy ? o1.re : o0.re, t.cy ? o1.im : o0.im};
            }
          }
        } else {
          // pruned: only the N_g target values of each column, as direct sums in double
          for (int w = tid; w < zg * H * NL; w += NT) {
            const int kx = w % H, yy = (w / H) % NL, zz = w / (H * NL);
            const int Y = (2 + t.cy) * NG - EXT + yy;
            const cplx<T>* col = slab + size_t(zz) * ENT + kx;
            cplx<double> acc = {0.0, 0.0};
            int mi = 0;
#pragma unroll 8
            for (int ky = 0; ky < n; ++ky) {
              const cplx<double> tv = s_tw[mi];
              const cplx<T> f = col[size_t(ky) * H];
              acc.re = fma(double(f.re), tv.re, fma(-double(f.im), tv.im, acc.re));
              acc.im = fma(double(f.re), tv.im, fma(double(f.im), tv.re, acc.im));
              mi += Y;
              if (mi >= n) mi -= n;
            }
            red[(size_t(zp + z0 + zz) * NL + yy) * H + kx] = acc;
          }
        }
        __syncthreads();
      }
    }
    // x^-1 (Hermitian half spectrum): out = sum_k w_k Re(F_k e^{+2 pi i k X / n}), w_k = 1 at
    // k = 0 and n/2, 2 otherwise; X = (2 + c_x) N_g - EXT + xx
    const int Xt = (2 + t.cx) * NG - EXT;
    if constexpr (STRICT) {
      // the same sums in float-float: each product of a float spectrum value and a float-float
      // twiddle formed exactly to float-float precision, the terms added with renormalisation
      ff32* s_outf = reinterpret_cast<ff32*>(s_out);
      for (int q = tid; q < ML; q += NT) {
        const int xx = q % NL, row = q / NL;
        const int X = Xt + xx;
        const cplx<typename S::RedT>* F = red + size_t(row) * H;
        ff32 acc = {0.0f, 0.0f};
        int m = 0;
        for (int k = 0; k < H; ++k) {
          const float4 w = s_twf[m];
          ff32 v = ff_add(ff_mul(float(F[k].re), ff32{w.x, w.z}),
                          ff_neg(ff_mul(float(F[k].im), ff32{w.y, w.w})));
          if (!(k == 0 || k == n / 2)) v = {2.0f * v.hi, 2.0f * v.lo};
          acc = ff_add(acc, v);
          m += X;
          if (m >= n) m -= n;
        }
        s_outf[q] = acc;
      }
      __syncthreads();
      // result = mean (a float pair, per target) + zero-mean gridlet
      ff32* s_redf = reinterpret_cast<ff32*>(s_red);
      ff32 part = {0.0f, 0.0f};
      for (int e = tid; e < ML; e += NT) part = ff_add(part, s_outf[e]);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1)
        part = ff_add(part, ff32{__shfl_xor(part.hi, o, 64), __shfl_xor(part.lo, o, 64)});
      if ((tid & 63) == 0) s_redf[tid >> 6] = part;
      __syncthreads();
      ff32 sum = {0.0f, 0.0f};
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) sum = ff_add(sum, s_redf[w]);
      const ff32 mean = ff_div(sum, ML);
      for (int e = tid; e < ML; e += NT)
        a.local[size_t(t.g) * ML + e] = ff_add(s_outf[e], ff_neg(mean)).hi;
      if (tid == 0) reinterpret_cast<ff32*>(a.m2l_mean)[t.g] = mean;
    } else {
      for (int q = tid; q < ML; q += NT) {
        const int xx = q % NL, row = q / NL;
        const int X = Xt + xx;
        const cplx<typename S::RedT>* F = red + size_t(row) * H;
        double acc = 0.0;
        int m = 0;
        for (int k = 0; k < H; ++k) {
          const cplx<double> f = {double(F[k].re), double(F[k].im)};
          const cplx<double> w = s_tw[m];
          const double v = f.re * w.re - f.im * w.im;
          acc += (k == 0 || k == n / 2) ? v : 2.0 * v;
          m += X;
          if (m >= n) m -= n;
        }
        s_out[q] = acc;
      }
      __syncthreads();
      // result = mean (double, per target) + zero-mean gridlet (T)
      double part = 0.0;
      for (int e = tid; e < ML; e += NT) part += s_out[e];
      part = wave_sum(part);
      if ((tid & 63) == 0) s_red[tid >> 6] = part;
      __syncthreads();
      double mean = 0.0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) mean += s_red[w];
      mean *= 1.0 / ML;
      for (int e = tid; e < ML; e += NT) a.local[size_t(t.g) * ML + e] = T(s_out[e] - mean);
      if (tid == 0) a.m2l_mean[t.g] = mean;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// The transform shared by the children of one split parent. Every child's interaction zone lies
// in the parent's 6^3 block; the 152 block cubes outside the central 4^3 are in the zone of all
// 8 children. One workgroup per parent runs the z-slab scheme over those cubes for each half cz
// of the children (target z window (2 + cz) N_g .. (3 + cz) N_g - 1, the accumulators of one
// window per pass), then the inverse y transform keeping both children's y windows, then for
// each existing child the inverse x transform, its mean and its zero-mean gridlet. The other 37
// cubes of each child's zone are added afterwards, cell by cell.
// ---------------------------------------------------------------------------------------------
template <typename T, int NG>
struct ParentShape {
  using S = SlabShape<T, NG>;
  static constexpr size_t red_bytes = size_t(NG) * 2 * NG * S::H * sizeof(cplx<T>) +
                                      size_t(S::M) * 8 + size_t(S::n) * sizeof(cplx<double>);
  static constexpr bool fits = !S::narrow && S::slab_bytes + red_bytes + 216 * 4 + 64 <= 150 * 1024;
};

template <typename T, int NG>
__global__ __launch_bounds__(kSlabThreads) void k_m2l_parent(M2LArgs<T> a) {
  using S = SlabShape<T, NG>;
  constexpr int n = S::n, H = S::H, M = S::M, NT = S::NT, D = S::D, PER = S::PER, ENT = S::ENT;
  static_assert(ParentShape<T, NG>::fits, "parent buffers exceed the LDS budget");
  static_assert(S::ZB >= NG, "the slab buffer holds the N_g accumulated planes");
  __shared__ int s_src[216];
  __shared__ int s_kid[8];
  __shared__ int s_off[kMaxLevels + 1];
  __shared__ __align__(16) cplx<T> slab[S::ZB * n * H];
  __shared__ cplx<T> red[NG * 2 * NG * H];  // after y^-1: [Z][Y, both children's windows][kx]
  __shared__ double s_out[M];
  __shared__ double s_red[NT / 64];
  __shared__ cplx<double> s_tw[n];  // e^{+2 pi i m / n}
  const int tid = threadIdx.x;
  if (tid <= kMaxLevels) s_off[tid] = a.level_off[tid];
  for (int m = tid; m < n; m += NT) {
    double sv, cv;
    sincospi(2.0 * m / n, &sv, &cv);
    s_tw[m] = {cv, sv};
  }

  const int xcd = blockIdx.x & 7, per = gridDim.x >> 3, jb = blockIdx.x >> 3;
  const int p_begin = int((int64_t(a.nparents) * xcd) / 8);
  const int p_end = int((int64_t(a.nparents) * (xcd + 1)) / 8);

  for (int pi_ = p_begin + jb; pi_ < p_end; pi_ += per) {
    __syncthreads();
    const int par = a.plist[pi_];
    const int l = level_of(par, s_off, a.nlevels) + 1;  // the children's level (>= 2)
    if (tid < 216) {
      const int bx = tid % 6, by = (tid / 6) % 6, bz = tid / 36;
      const bool central = bx >= 1 && bx <= 4 && by >= 1 && by <= 4 && bz >= 1 && bz <= 4;
      s_src[tid] = central ? -1 : a.blocks[size_t(par - a.first_parent) * 216 + tid];
    }
    if (tid < 8) s_kid[tid] = a.child8[size_t(par) * 8 + tid];
    __syncthreads();
    const T* gtab = a.gxy + size_t(l - 2) * D * H * H;

    for (int cz = 0; cz < 2; ++cz) {
      // block-uniform: every thread reads the same child ids
      if (s_kid[4 * cz] < 0 && s_kid[4 * cz + 1] < 0 && s_kid[4 * cz + 2] < 0 &&
          s_kid[4 * cz + 3] < 0)
        continue;
      T pr[PER][NG], pim[PER][NG];
      slab_sum<T, NG>(a, s_src, slab, gtab, (2 + cz) * NG, s_tw, pr, pim);
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const int e = tid + NT * r;
        if (e < ENT) {
#pragma unroll
          for (int zz = 0; zz < NG; ++zz) slab[size_t(zz) * ENT + e] = {pr[r][zz], pim[r][zz]};
        }
      }
      __syncthreads();
      // y^-1: red[Z][Y][kx], Y = 2 N_g + yy for yy < 2 N_g (the windows of cy = 0 and 1)
      for (int w = tid; w < NG * H; w += NT) {
        const int kx = w % H, zz = w / H;
        const cplx<T>* col = slab + size_t(zz) * ENT + kx;
        cplx<T> in[n], out[n];
#pragma unroll
        for (int y = 0; y < n; ++y) in[y] = col[size_t(y) * H];
        fft<n, +1>(in, out);
#pragma unroll
        for (int yy = 0; yy < 2 * NG; ++yy) red[(size_t(zz) * 2 * NG + yy) * H + kx] = out[2 * NG + yy];
      }
      __syncthreads();
      for (int c = 4 * cz; c < 4 * cz + 4; ++c) {
        const int g = s_kid[c];
        if (g < 0) continue;  // block-uniform
        const int cx = c & 1, cy = (c >> 1) & 1;
        // x^-1 (Hermitian half spectrum) in double: out = sum_k w_k Re(F_k e^{+2 pi i k X / n}),
        // w_k = 1 at k = 0 and n/2, 2 otherwise; X = (2 + c_x) N_g + xx
        const int Xt = (2 + cx) * NG;
        for (int q = tid; q < M; q += NT) {
          const int xx = q % NG, yy = (q / NG) % NG, zz = q / (NG * NG);
          const int X = Xt + xx;
          const cplx<T>* F = red + (size_t(zz) * 2 * NG + cy * NG + yy) * H;
          double acc = 0.0;
          int m = 0;
          for (int k = 0; k < H; ++k) {
            const cplx<double> f = {double(F[k].re), double(F[k].im)};
            const cplx<double> w = s_tw[m];
            const double v = f.re * w.re - f.im * w.im;
            acc += (k == 0 || k == n / 2) ? v : 2.0 * v;
            m += X;
            if (m >= n) m -= n;
          }
          s_out[q] = acc;
        }
        __syncthreads();
        double part = 0.0;
        for (int e = tid; e < M; e += NT) part += s_out[e];
        part = wave_sum(part);
        if ((tid & 63) == 0) s_red[tid >> 6] = part;
        __syncthreads();
        double mean = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) mean += s_red[w];
        mean *= 1.0 / M;
        for (int e = tid; e < M; e += NT) a.local[size_t(g) * M + e] = T(s_out[e] - mean);
        if (tid == 0) a.m2l_mean[g] = mean;
        __syncthreads();  // s_out and s_red are reused by the next child
      }
    }
  }
}

// Which kernel serves (T, N_g): from N_g = 4 on the z-slab kernel (both precisions; from N_g = 6
// in FP64 one workgroup per CU fits); below N_g = 4 the whole-grid kernel with its stage in LDS
// (at N_g = 4 in FP32 that stage would hold 104 KB, one workgroup per CU).
template <typename T, int NG>
constexpr int m2l_kind() {
  if constexpr (NG >= 4) {
    static_assert(SlabShape<T, NG>::fits, "z-slab buffers exceed the LDS budget");
    return 1;
  } else {
    static_assert(M2LShape<T, NG>::lds, "whole-grid stage exceeds the LDS budget");
    return 0;
  }
}

// resident workgroups of the z-slab kernel on 256 CUs
constexpr int kSlabGrid = 256 * kSlabPerCU;

// Workgroups of a source-to-target launch (the kernels keep every per-target buffer on the CU;
// there is no workspace in device memory).
int m2l_workspace_slots(int prec, int ng, size_t* bytes_per_slot) {
  *bytes_per_slot = 0;
  (void)prec;
  return ng >= 4 ? kSlabGrid : 8 * 256;
}

template <typename T, int NG>
static void m2l_t(Plan& p, hipStream_t s) {
  if (p.nlevels <= 2) return;
  M2LArgs<T> a;
  a.first_target = p.level_off[2];
  a.ntargets = int(p.ncells) - p.level_off[2];
  if (a.ntargets <= 0) return;
  a.nlevels = p.nlevels;
  a.depth = p.depth;
  a.level_off = p.dlev.as<int>() + kLevOff;
  a.coord = p.ccoord.as<int>();
  a.parent = p.cparent.as<int>();
  a.blocks = p.blocks.as<int>();
  a.first_parent = p.blocks_first;
  a.gridlet = p.gridlet.as<T>();
  a.local = p.local.as<T>();
  a.m2l_mean = p.m2l_mean.as<double>();
  a.ghat = p.tab.ghat.as<T>();
  a.gxy = p.tab.gxy.as<T>();
  a.lo0 = p.prob.box_lo[0];
  a.lo1 = p.prob.box_lo[1];
  a.lo2 = p.prob.box_lo[2];
  a.size = p.prob.box_size;
  int grid = ((a.ntargets + 7) / 8) * 8;
  if (grid > p.m2l_slots) grid = p.m2l_slots;
  p.m2l_split = m2l_kind<T, NG>() == 1;
  p.m2l_mean_ff = false;
  if constexpr (m2l_kind<T, NG>() == 1) {
    if constexpr (sizeof(T) == 4 && (NG == 4 || NG == 6)) {
      if (p.fp32_strict) {
        a.twff = p.tab.twff.as<float4>();
        p.m2l_mean_ff = true;
        if (p.ext) k_m2l_slab<T, NG, 1, true><<<grid, SlabShape<T, NG, 1>::NT, 0, s>>>(a);
        else k_m2l_slab<T, NG, 0, true><<<grid, SlabShape<T, NG>::NT, 0, s>>>(a);
        HPM_LAUNCH_CHECK();
        return;
      }
    }
    if (p.ext) {
      if constexpr (NG == 4 || NG == 6) k_m2l_slab<T, NG, 1><<<grid, SlabShape<T, NG, 1>::NT, 0, s>>>(a);
      else fail(HPM_ERR_UNSUPPORTED, "no extended padded-grid kernel for this gridlet");
    } else {
      k_m2l_slab<T, NG, 0><<<grid, SlabShape<T, NG>::NT, 0, s>>>(a);
    }
  } else {
    if (p.ext) fail(HPM_ERR_UNSUPPORTED, "no extended padded-grid kernel for this gridlet");
    k_m2l<T, NG><<<grid, 256, 0, s>>>(a);
  }
  HPM_LAUNCH_CHECK();
}

// The per-parent shared transform over the outer cubes of every split parent's block; it writes
// each child's result as (mean, zero-mean gridlet), which the cell-by-cell pass over the central
// cubes then adds to.
template <typename T, int NG>
static void parents_t(Plan& p, hipStream_t s) {
  if constexpr (!ParentShape<T, NG>::fits) {
    fail(HPM_ERR_UNSUPPORTED, "no shared-transform kernel for this gridlet");
  } else {
    p.m2l_split = true;
    if (p.nlevels <= 2) return;
    M2LArgs<T> a{};
    a.nparents = p.cell_pbeg[p.nlevels - 1];
    if (a.nparents <= 0) return;
    const int64_t first = p.level_off[1], last = p.level_off[p.nlevels - 1];
    if (p.cell_plist.bytes < size_t(a.nparents) * 4 ||
        p.blocks.bytes < size_t(last - first) * 216 * 4 || p.blocks_first != first ||
        p.local.bytes < size_t(p.ncells) * SlabShape<T, NG>::M * sizeof(T))
      fail(HPM_ERR_DEVICE, "shared-transform buffers inconsistent with the tree");
    a.nlevels = p.nlevels;
    a.depth = p.depth;
    a.level_off = p.dlev.as<int>() + kLevOff;
    a.blocks = p.blocks.as<int>();
    a.first_parent = p.blocks_first;
    a.gridlet = p.gridlet.as<T>();
    a.local = p.local.as<T>();
    a.m2l_mean = p.m2l_mean.as<double>();
    a.gxy = p.tab.gxy.as<T>();
    a.size = p.prob.box_size;
    a.plist = p.cell_plist.as<int>();
    a.child8 = p.child8.as<int>();
    int grid = ((a.nparents + 7) / 8) * 8;
    if (grid > kSlabGrid) grid = kSlabGrid;
    k_m2l_parent<T, NG><<<grid, SlabShape<T, NG>::NT, 0, s>>>(a);
    HPM_LAUNCH_CHECK();
  }
}

void launch_m2l_parents(Plan& p, hipStream_t s) {
  if (p.prec == HPM_F32) {
    switch (p.ng) {
      case 2: parents_t<float, 2>(p, s); break;
      case 3: parents_t<float, 3>(p, s); break;
      case 4: parents_t<float, 4>(p, s); break;
      case 6: parents_t<float, 6>(p, s); break;
      default: fail(HPM_ERR_UNSUPPORTED, "no shared-transform kernel for this gridlet");
    }
  } else {
    switch (p.ng) {
      case 2: parents_t<double, 2>(p, s); break;
      case 3: parents_t<double, 3>(p, s); break;
      case 4: parents_t<double, 4>(p, s); break;
      case 6: parents_t<double, 6>(p, s); break;
      default: fail(HPM_ERR_UNSUPPORTED, "no shared-transform kernel for this gridlet");
    }
  }
}

void launch_m2l(Plan& p, hipStream_t s) {
  if (p.prec == HPM_F32) {
    switch (p.ng) {
      case 2: m2l_t<float, 2>(p, s); break;
      case 3: m2l_t<float, 3>(p, s); break;
      case 4: m2l_t<float, 4>(p, s); break;
      case 6: m2l_t<float, 6>(p, s); break;
      case 8: m2l_t<float, 8>(p, s); break;
    }
  } else {
    switch (p.ng) {
      case 2: m2l_t<double, 2>(p, s); break;
      case 3: m2l_t<double, 3>(p, s); break;
      case 4: m2l_t<double, 4>(p, s); break;
      case 6: m2l_t<double, 6>(p, s); break;
      case 8: m2l_t<double, 8>(p, s); break;
    }
  }
}

}  // namespace hpm
