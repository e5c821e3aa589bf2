// Down-sweep and leaves: parent-to-child translation (Sec. 2.4, Eq. 6-7), the far field at the
// particles (Eq. 7 and its gradient) and the near-zone direct sum (Sec. 1), plus a brute-force
// direct sum used as the accuracy reference.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "hpm_internal.h"

namespace hpm {

// Phi^C_q += sum_p Phi^P_p l_p((a^C + x_q)/2): the transpose of the separable child-to-parent
// matrix, one workgroup per child cell of level "off.."; its parent is at level >= 2.
template <typename T, int NG>
__global__ __launch_bounds__(256) void k_l2l(int off, const int* __restrict__ parent,
                                             const int* __restrict__ coord, const T* __restrict__ t1,
                                             T* __restrict__ local) {
  constexpr int M = NG * NG * NG;
  __shared__ T s_in[M], s_a[M], s_b[M];
  __shared__ T s_t[2][NG][NG];
  const int g = off + blockIdx.x;
  const int tid = threadIdx.x;
  const int P = parent[g];
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
  for (int e = tid; e < M; e += 256) {  // out[qz][qy][qx]
    const int qx = e % NG, qy = (e / NG) % NG, qz = e / (NG * NG);
    T acc = T(0);
#pragma unroll
    for (int p = 0; p < NG; ++p) acc += s_t[az][p][qz] * s_b[(p * NG + qy) * NG + qx];
    local[size_t(g) * M + e] += acc;
  }
}

template <typename T>
struct LeafArgs {
  int n;
  const int* leaves;
  const int* level_off;
  int nlevels;
  int depth;
  const int* coord;
  const int* pb;
  const int* pe;
  const int* nbr27;
  const uint32_t* keys;
  const int* perm;
  const T* xs;
  const T* ys;
  const T* zs;
  const T* ms;
  const T* local;
  T* phi;
  T* ax;
  T* ay;
  T* az;
  double lo0, lo1, lo2, size;
  T gconst;
  T eps2;
};

template <typename T>
__device__ __forceinline__ T inv_sqrt(T x) {
  if constexpr (sizeof(T) == 4) return rsqrtf(x);
  else return 1.0 / sqrt(x);
}

// One wave per leaf. Near zone: the 27 level-l cubes around the leaf, each a contiguous range of
// sorted particles (a real cell's range, or the part of a coarser leaf inside that cube). Source
// particles are staged 64 at a time in LDS; when the leaf has fewer than 64 particles the lanes
// split the sources into groups and the partial sums are combined with wave shuffles. The
// potential is accumulated with Kahan compensation; near and far parts are added last.
template <typename T, int NG>
__global__ __launch_bounds__(64) void k_leaf(LeafArgs<T> a) {
  constexpr int M = NG * NG * NG;
  __shared__ int s_off[kMaxLevels + 1];
  __shared__ int s_rb[27], s_re[27], s_pre[28];
  __shared__ T s_x[64], s_y[64], s_z[64], s_m[64];
  __shared__ int s_id[64];
  __shared__ T s_phi[M];
  const int lane = threadIdx.x;
  if (lane <= kMaxLevels) s_off[lane] = a.level_off[lane];
  __syncthreads();
  const int g = a.leaves[blockIdx.x];
  const int l = level_of(g, s_off, a.nlevels);
  const int pc = a.coord[g];
  const int tx = coord_x(pc), ty = coord_y(pc), tz = coord_z(pc);
  const int pb = a.pb[g], pe = a.pe[g];
  const int K = pe - pb;
  if (lane < 27) {
    const int e = a.nbr27[g * 27 + lane];
    int rb = 0, re = 0;
    if (e >= 0) {
      rb = a.pb[e];
      re = a.pe[e];
    } else if (e <= -2) {
      const int c = -2 - e;
      const int qx = tx + lane % 3 - 1, qy = ty + (lane / 3) % 3 - 1, qz = tz + lane / 9 - 1;
      const uint32_t key = morton3(uint32_t(qx), uint32_t(qy), uint32_t(qz), l);
      const int shift = 3 * (a.depth - l);
      rb = lower_bound_u32(a.keys, a.pb[c], a.pe[c], key << shift);
      re = lower_bound_u32(a.keys, rb, a.pe[c], (key + 1u) << shift);
    }
    s_rb[lane] = rb;
    s_re[lane] = re;
  }
  if (l >= 2)
    for (int e = lane; e < M; e += 64) s_phi[e] = a.local[size_t(g) * M + e];
  __syncthreads();
  if (lane == 0) {
    int acc = 0;
    for (int r = 0; r < 27; ++r) {
      s_pre[r] = acc;
      acc += s_re[r] - s_rb[r];
    }
    s_pre[27] = acc;
  }
  __syncthreads();
  const int S = s_pre[27];
  int kp = 1;
  while (kp < K && kp < 64) kp <<= 1;
  const int G = 64 / kp;
  const int tl = lane % kp, grp = lane / kp;
  const double L = a.size / double(1 << l);
  const T cxc = T(a.lo0 + (tx + 0.5) * L), cyc = T(a.lo1 + (ty + 0.5) * L), czc = T(a.lo2 + (tz + 0.5) * L);
  const T invL = T(1.0 / L);

  for (int t0 = 0; t0 < K; t0 += kp) {
    const int i = pb + t0 + tl;
    const bool valid = (t0 + tl) < K;
    T xi = T(0), yi = T(0), zi = T(0);
    if (valid) {
      xi = a.xs[i];
      yi = a.ys[i];
      zi = a.zs[i];
    }
    T ph = T(0), phc = T(0), fx = T(0), fy = T(0), fz = T(0);
    for (int s0 = 0; s0 < S; s0 += 64) {
      const int sidx = s0 + lane;
      __syncthreads();
      if (sidx < S) {
        int r = 0;
        while (r < 26 && s_pre[r + 1] <= sidx) ++r;
        const int j = s_rb[r] + (sidx - s_pre[r]);
        s_x[lane] = a.xs[j];
        s_y[lane] = a.ys[j];
        s_z[lane] = a.zs[j];
        s_m[lane] = a.ms[j];
        s_id[lane] = j;
      }
      __syncthreads();
      const int cnt = min(64, S - s0);
      if (valid) {
        for (int e = grp; e < cnt; e += G) {
          const T dx = xi - s_x[e], dy = yi - s_y[e], dz = zi - s_z[e];
          const T r2 = dx * dx + dy * dy + dz * dz + a.eps2;
          const T inv = (s_id[e] == i) ? T(0) : inv_sqrt(r2);
          const T mi = s_m[e] * inv;
          const T mi3 = mi * inv * inv;
          // Kahan: ph += -m/r
          const T yv = -mi - phc;
          const T tv = ph + yv;
          phc = (tv - ph) - yv;
          ph = tv;
          fx -= mi3 * dx;
          fy -= mi3 * dy;
          fz -= mi3 * dz;
        }
      }
    }
    // combine the source groups (compensated for the potential)
    T phs = ph, phe = -phc;
    for (int o = kp; o < 64; o <<= 1) {
      const T ophs = __shfl_xor(phs, o, 64), ophe = __shfl_xor(phe, o, 64);
      const T s = phs + ophs;
      const T bb = s - phs;
      phe += ophe + ((phs - (s - bb)) + (ophs - bb));
      phs = s;
      fx += __shfl_xor(fx, o, 64);
      fy += __shfl_xor(fy, o, 64);
      fz += __shfl_xor(fz, o, 64);
    }
    if (valid && grp == 0) {
      T pfar = T(0), gx = T(0), gy = T(0), gz = T(0);
      if (l >= 2) {
        T lx[NG], dlx[NG], ly[NG], dly[NG], lz[NG], dlz[NG];
        lagrange_basis_d<NG>((xi - cxc) * invL, lx, dlx);
        lagrange_basis_d<NG>((yi - cyc) * invL, ly, dly);
        lagrange_basis_d<NG>((zi - czc) * invL, lz, dlz);
#pragma unroll
        for (int k = 0; k < NG; ++k) {
#pragma unroll
          for (int j = 0; j < NG; ++j) {
            T r0 = T(0), r1 = T(0);
#pragma unroll
            for (int q = 0; q < NG; ++q) {
              const T v = s_phi[(k * NG + j) * NG + q];
              r0 += lx[q] * v;
              r1 += dlx[q] * v;
            }
            pfar += lz[k] * ly[j] * r0;
            gx += lz[k] * ly[j] * r1;
            gy += lz[k] * dly[j] * r0;
            gz += dlz[k] * ly[j] * r0;
          }
        }
      }
      // total = G * near + far, the near part carried as (phs, phe)
      const T gn = a.gconst;
      const T near_hi = gn * phs;
      const T near_lo = fma(gn, phs, -near_hi) + gn * phe;
      const T s = near_hi + pfar;
      const T bb = s - near_hi;
      const T err = (near_hi - (s - bb)) + (pfar - bb);
      const int o = a.perm[i];
      if (o < 0 || o >= a.n) continue;
      a.phi[o] = s + (err + near_lo);
      a.ax[o] = gn * fx - gx * invL;
      a.ay[o] = gn * fy - gy * invL;
      a.az[o] = gn * fz - gz * invL;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_direct(int n, const T* x, const T* y, const T* z, const T* m,
                                                const int* targets, double G, double eps2, double* phi,
                                                double* ax, double* ay, double* az) {
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
    const double mi = double(m[j]) * inv;
    const double mi3 = mi * inv * inv;
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
  k_l2l<T, NG><<<cnt, 256, 0, s>>>(off, p.cparent.as<int>(), p.ccoord.as<int>(), p.tab.m2m.as<T>(),
                                   p.local.as<T>());
  HPM_LAUNCH_CHECK();
}

template <typename T, int NG>
static void leaf_t(Plan& p, void* phi, void* ax, void* ay, void* az, hipStream_t s) {
  if (p.nleaves <= 0) return;
  LeafArgs<T> a;
  a.n = int(p.n);
  a.leaves = p.leaves.as<int>();
  a.level_off = p.dlevel.as<int>();
  a.nlevels = p.nlevels;
  a.depth = p.depth;
  a.coord = p.ccoord.as<int>();
  a.pb = p.cpb.as<int>();
  a.pe = p.cpe.as<int>();
  a.nbr27 = p.nbr27.as<int>();
  a.keys = p.keys.as<uint32_t>();
  a.perm = p.perm.as<int>();
  a.xs = p.xs.as<T>();
  a.ys = p.ys.as<T>();
  a.zs = p.zs.as<T>();
  a.ms = p.ms.as<T>();
  a.local = p.local.as<T>();
  a.phi = (T*)phi;
  a.ax = (T*)ax;
  a.ay = (T*)ay;
  a.az = (T*)az;
  a.lo0 = p.prob.box_lo[0];
  a.lo1 = p.prob.box_lo[1];
  a.lo2 = p.prob.box_lo[2];
  a.size = p.prob.box_size;
  a.gconst = T(p.prob.gconst);
  a.eps2 = T(p.prob.softening * p.prob.softening);
  k_leaf<T, NG><<<int(p.nleaves), 64, 0, s>>>(a);
  HPM_LAUNCH_CHECK();
}

#define HPM_DISPATCH_NG(FN, ...)                                                   \
  do {                                                                             \
    if (p.prec == HPM_F32) {                                                       \
      switch (p.ng) {                                                              \
        case 2: FN<float, 2>(__VA_ARGS__); break;                                  \
        case 3: FN<float, 3>(__VA_ARGS__); break;                                  \
        case 4: FN<float, 4>(__VA_ARGS__); break;                                  \
        case 6: FN<float, 6>(__VA_ARGS__); break;                                  \
        case 8: FN<float, 8>(__VA_ARGS__); break;                                  \
      }                                                                            \
    } else {                                                                       \
      switch (p.ng) {                                                              \
        case 2: FN<double, 2>(__VA_ARGS__); break;                                 \
        case 3: FN<double, 3>(__VA_ARGS__); break;                                 \
        case 4: FN<double, 4>(__VA_ARGS__); break;                                 \
        case 6: FN<double, 6>(__VA_ARGS__); break;                                 \
        case 8: FN<double, 8>(__VA_ARGS__); break;                                 \
      }                                                                            \
    }                                                                              \
  } while (0)

void launch_l2l(Plan& p, int level, hipStream_t s) { HPM_DISPATCH_NG(l2l_t, p, level, s); }
void launch_leaf(Plan& p, void* phi, void* ax, void* ay, void* az, hipStream_t s) {
  HPM_DISPATCH_NG(leaf_t, p, phi, ax, ay, az, s);
}

void launch_direct_sum(int prec, int64_t n, const void* x, const void* y, const void* z,
                       const void* m, int64_t nt, const int32_t* targets, double G, double eps,
                       double* phi, double* ax, double* ay, double* az, hipStream_t s) {
  if (nt <= 0) return;
  if (prec == HPM_F32)
    k_direct<float><<<int(nt), 256, 0, s>>>(int(n), (const float*)x, (const float*)y,
                                            (const float*)z, (const float*)m, targets, G, eps * eps,
                                            phi, ax, ay, az);
  else
    k_direct<double><<<int(nt), 256, 0, s>>>(int(n), (const double*)x, (const double*)y,
                                             (const double*)z, (const double*)m, targets, G,
                                             eps * eps, phi, ax, ay, az);
  HPM_LAUNCH_CHECK();
}

}  // namespace hpm
