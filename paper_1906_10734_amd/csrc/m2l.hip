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
// The line buffer ("stage", layout [z < 6N_g][y < n][kx <= n/2] complex) lives in LDS when it
// fits, else in a per-workgroup slice of global memory. Cubes of the interaction zone that are
// not cells of the tree but lie inside a coarser leaf get their effective masses here, from the
// particles inside them (Lagrange weights, the closed form of Eq. 5).
#include <hip/hip_runtime.h>

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
  const int* flags;
  const int* child8;
  const int* nbr27;
  const int* pb;
  const int* pe;
  const uint32_t* keys;
  const T* xs;
  const T* ys;
  const T* zs;
  const T* ms;
  const T* gridlet;
  T* local;
  const T* ghat;
  cplx<T>* work;
  double lo0, lo1, lo2, size;
};

constexpr int fold_k(int k, int n) { return k <= n / 2 ? k : n - k; }

template <typename T, int NG>
__global__ __launch_bounds__(256) void k_m2l(M2LArgs<T> a) {
  using S = M2LShape<T, NG>;
  constexpr int n = S::n, H = S::H, W = S::W, M = S::M;
  __shared__ int s_src[216];
  __shared__ int s_vb[216];
  __shared__ int s_ve[216];
  __shared__ int s_off[kMaxLevels + 1];
  cplx<T>* stage;
  if constexpr (S::lds) {
    __shared__ cplx<T> s_stage[S::elems];
    stage = s_stage;
  } else {
    stage = a.work + size_t(blockIdx.x) * S::elems;
  }
  const int tid = threadIdx.x;
  if (tid <= kMaxLevels) s_off[tid] = a.level_off[tid];

  // The 8 XCDs take contiguous chunks of the Morton-ordered targets (neighbouring targets
  // share most of their interaction zones, so their gridlets stay in the XCD's L2).
  const int xcd = blockIdx.x & 7, per = gridDim.x >> 3, j = blockIdx.x >> 3;
  const int t_begin = int((int64_t(a.ntargets) * xcd) / 8);
  const int t_end = int((int64_t(a.ntargets) * (xcd + 1)) / 8);

  for (int t = t_begin + j; t < t_end; t += per) {
    const int g = a.first_target + t;
    __syncthreads();
    const int l = level_of(g, s_off, a.nlevels);
    const int pc = a.coord[g];
    const int tx = coord_x(pc), ty = coord_y(pc), tz = coord_z(pc);
    const int cx = tx & 1, cy = ty & 1, cz = tz & 1;
    const int par = a.parent[g];
    const double L = a.size / double(1 << l);

    // ---- resolve the 216 cubes of the block -------------------------------------------------
    if (tid < 216) {
      const int bx = tid % 6, by = (tid / 6) % 6, bz = tid / 36;
      int src = -1, vb = 0, ve = 0;
      const bool near = abs(bx - 2 - cx) <= 1 && abs(by - 2 - cy) <= 1 && abs(bz - 2 - cz) <= 1;
      if (!near) {
        const int e = a.nbr27[par * 27 + (bx >> 1) + 3 * (by >> 1) + 9 * (bz >> 1)];
        const int oct = (bx & 1) | ((by & 1) << 1) | ((bz & 1) << 2);
        int coarse = -1;
        if (e >= 0) {
          if (a.flags[e] & 1) src = a.child8[e * 8 + oct];
          else coarse = e;
        } else if (e <= -2) {
          coarse = -2 - e;
        }
        if (coarse >= 0) {
          const int qx = 2 * ((tx >> 1) - 1) + bx, qy = 2 * ((ty >> 1) - 1) + by,
                    qz = 2 * ((tz >> 1) - 1) + bz;
          const uint32_t key = morton3(uint32_t(qx), uint32_t(qy), uint32_t(qz), l);
          const int shift = 3 * (a.depth - l);
          const int cb = a.pb[coarse], ce = a.pe[coarse];
          vb = lower_bound_u32(a.keys, cb, ce, key << shift);
          ve = lower_bound_u32(a.keys, vb, ce, (key + 1u) << shift);
          src = (ve > vb) ? -2 : -1;
        }
      }
      s_src[tid] = src;
      s_vb[tid] = vb;
      s_ve[tid] = ve;
    }
    __syncthreads();

    // ---- x: gather two rows, real-to-complex --------------------------------------------------
    for (int w = tid; w < W * W / 2; w += blockDim.x) {
      const int r0 = 2 * w;
      const int y0 = r0 % W, zr = r0 / W;  // rows (y0, zr) and (y0 + 1, zr)
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
          const int s = bx + 6 * (by + 6 * bz);
          const int src = s_src[s];
          T v[NG];
#pragma unroll
          for (int i = 0; i < NG; ++i) v[i] = T(0);
          if (src >= 0) {
            const T* gsrc = a.gridlet + size_t(src) * M + (kz * NG + jy) * NG;
#pragma unroll
            for (int i = 0; i < NG; ++i) v[i] = gsrc[i];
          } else if (src == -2) {
            const int qx = 2 * ((tx >> 1) - 1) + bx, qy = 2 * ((ty >> 1) - 1) + by,
                      qz = 2 * ((tz >> 1) - 1) + bz;
            const T ccx = T(a.lo0 + (qx + 0.5) * L), ccy = T(a.lo1 + (qy + 0.5) * L),
                    ccz = T(a.lo2 + (qz + 0.5) * L);
            const T invL = T(1.0 / L);
            for (int p = s_vb[s]; p < s_ve[s]; ++p) {
              T lx[NG], ly[NG], lz[NG];
              lagrange_basis<NG>((a.xs[p] - ccx) * invL, lx);
              lagrange_basis<NG>((a.ys[p] - ccy) * invL, ly);
              lagrange_basis<NG>((a.zs[p] - ccz) * invL, lz);
              T wyz = a.ms[p];
#pragma unroll
              for (int q = 0; q < NG; ++q) wyz = (q == jy) ? wyz * ly[q] : wyz;
              T wz = T(0);
#pragma unroll
              for (int q = 0; q < NG; ++q) wz = (q == kz) ? lz[q] : wz;
              wyz *= wz;
#pragma unroll
              for (int i = 0; i < NG; ++i) v[i] += wyz * lx[i];
            }
          }
#pragma unroll
          for (int i = 0; i < NG; ++i) {
            if (half == 0) line[bx * NG + i].re = v[i];
            else line[bx * NG + i].im = v[i];
          }
        }
      }
      cplx<T> zf[n];
      fft<n, -1>(line, zf);
      cplx<T>* row0 = stage + (size_t(zr) * n + y0) * H;
      cplx<T>* row1 = row0 + H;
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const cplx<T> z1 = zf[k], z2 = zf[(n - k) % n];
        row0[k] = {T(0.5) * (z1.re + z2.re), T(0.5) * (z1.im - z2.im)};
        row1[k] = {T(0.5) * (z1.im + z2.im), T(0.5) * (z2.re - z1.re)};
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

int m2l_workspace_slots(int prec, int ng, size_t* bytes_per_slot) {
  size_t b = 0;
  bool lds = true;
#define HPM_SHAPE(TT, NN)                      \
  if (ng == NN) {                              \
    b = M2LShape<TT, NN>::bytes;               \
    lds = M2LShape<TT, NN>::lds;               \
  }
  if (prec == HPM_F32) {
    HPM_SHAPE(float, 2) HPM_SHAPE(float, 3) HPM_SHAPE(float, 4) HPM_SHAPE(float, 6) HPM_SHAPE(float, 8)
  } else {
    HPM_SHAPE(double, 2) HPM_SHAPE(double, 3) HPM_SHAPE(double, 4) HPM_SHAPE(double, 6) HPM_SHAPE(double, 8)
  }
#undef HPM_SHAPE
  *bytes_per_slot = lds ? 0 : b;
  if (lds) return 8 * 256;
  return b > (size_t(1) << 20) ? 1024 : 2048;
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
  a.level_off = p.dlevel.as<int>();
  a.coord = p.ccoord.as<int>();
  a.parent = p.cparent.as<int>();
  a.flags = p.cflags.as<int>();
  a.child8 = p.child8.as<int>();
  a.nbr27 = p.nbr27.as<int>();
  a.pb = p.cpb.as<int>();
  a.pe = p.cpe.as<int>();
  a.keys = p.keys.as<uint32_t>();
  a.xs = p.xs.as<T>();
  a.ys = p.ys.as<T>();
  a.zs = p.zs.as<T>();
  a.ms = p.ms.as<T>();
  a.gridlet = p.gridlet.as<T>();
  a.local = p.local.as<T>();
  a.ghat = p.tab.ghat.as<T>();
  a.work = p.m2l_work.as<cplx<T>>();
  a.lo0 = p.prob.box_lo[0];
  a.lo1 = p.prob.box_lo[1];
  a.lo2 = p.prob.box_lo[2];
  a.size = p.prob.box_size;
  int grid = ((a.ntargets + 7) / 8) * 8;
  if (grid > p.m2l_slots) grid = p.m2l_slots;
  k_m2l<T, NG><<<grid, 256, 0, s>>>(a);
  HPM_LAUNCH_CHECK();
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
