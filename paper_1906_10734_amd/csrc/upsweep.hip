// Up-sweep: leaf effective masses (Sec. 2.2, Eq. 2-5) and child-to-parent translation
// (Sec. 2.3).
//
// P2M is split as in Eq. (5): first the moments of each leaf at level >= 2 (one wave per leaf,
// moments in the tensor Legendre basis about the cell centre, so |phi_n| <= 1 and the sums are
// well conditioned in FP32), then M = B^phi Q for all leaves at once as a dense batched GEMM on
// the matrix cores (v_mfma_*_16x16x4 with FP32 or FP64 operands, so there is no precision loss).
// M2M applies the separable T^C = T1^{az} (x) T1^{ay} (x) T1^{ax} of every present child, one
// workgroup per parent, three LDS passes per child.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dev_common.h"
#include "hpm_internal.h"

namespace hpm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T>
__global__ void k_gather_masses(int n, const int* perm, const T* m, T* ms) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = perm[i];
  if (j >= 0 && j < n) ms[i] = m[j];
}

template <typename T>
struct P2MArgs {
  const int* leaves;
  const int* row_level;  // level of each row, or null: taken from the cell id
  int first;  // index of the first level>=2 leaf in the leaf list
  int count;
  const int* level_off;
  int nlevels;
  const int* coord;
  const int* pb;
  const int* pe;
  const T* xs;
  const T* ys;
  const T* zs;
  const T* ms;
  T* moments;  // [count][kpad]
  int kpad;
  double lo0, lo1, lo2, size;
};

template <typename T, int NG>
__global__ __launch_bounds__(64) void k_p2m_moments(P2MArgs<T> a) {
  constexpr int M = NG * NG * NG;
  constexpr int PER = (M + 63) / 64;
  __shared__ T s_b[3][64][NG];
  __shared__ int s_off[kMaxLevels + 1];
  const int lane = threadIdx.x;
  if (lane <= kMaxLevels) s_off[lane] = a.level_off[lane];
  __syncthreads();
  const int b = blockIdx.x;
  const int g = a.leaves[a.first + b];
  const int l = a.row_level ? a.row_level[b] : level_of(g, s_off, a.nlevels);
  const double L = a.size / double(1 << l);
  const int pc = a.coord[g];
  const T cx = T(a.lo0 + (coord_x(pc) + 0.5) * L);
  const T cy = T(a.lo1 + (coord_y(pc) + 0.5) * L);
  const T cz = T(a.lo2 + (coord_z(pc) + 0.5) * L);
  const T two_over_L = T(2.0 / L);
  const int pb = a.pb[g], pe = a.pe[g];
  T acc[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) acc[r] = T(0);
  for (int j0 = pb; j0 < pe; j0 += 64) {
    const int j = j0 + lane;
    T bx[NG], by[NG], bz[NG];
    T mj = T(0);
    if (j < pe) {
      legendre<NG>((a.xs[j] - cx) * two_over_L, bx);
      legendre<NG>((a.ys[j] - cy) * two_over_L, by);
      legendre<NG>((a.zs[j] - cz) * two_over_L, bz);
      mj = a.ms[j];
    } else {
#pragma unroll
      for (int k = 0; k < NG; ++k) bx[k] = by[k] = bz[k] = T(0);
    }
    // the mass goes into the x factor: each term is (m P_a(x)) P_b(y) P_c(z), evaluated left to right
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      s_b[0][lane][k] = mj * bx[k];
      s_b[1][lane][k] = by[k];
      s_b[2][lane][k] = bz[k];
    }
    __syncthreads();
    const int cnt = min(64, pe - j0);
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int nidx = lane + 64 * r;
      if (nidx < M) {
        const int nx = nidx % NG, ny = (nidx / NG) % NG, nz = nidx / (NG * NG);
        T s = acc[r];
        for (int jj = 0; jj < cnt; ++jj) s += s_b[0][jj][nx] * s_b[1][jj][ny] * s_b[2][jj][nz];
        acc[r] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int nidx = lane + 64 * r;
    if (nidx < a.kpad) a.moments[size_t(b) * a.kpad + nidx] = (nidx < M) ? acc[r] : T(0);
  }
  for (int nidx = lane + 64 * PER; nidx < a.kpad; nidx += 64) a.moments[size_t(b) * a.kpad + nidx] = T(0);
}

// gridlet[leaf][p] = sum_n Q[row][n] W[n][p] on the matrix cores. A workgroup takes 32 rows;
// each wave one 16-row tile and half of the 16-column tiles, so every A fragment feeds several
// independent accumulators. W passes through LDS in chunks of KC rows loaded by the whole
// workgroup at once (its loads are all in flight together), the A fragments of a chunk are
// loaded into registers ahead of the chunk's MFMAs.
// Operand layout of v_mfma_*_16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16]. The
// output rows differ by dtype (measured on gfx950): accumulator register v of lane l holds
// D[4*(l/16)+v][l%16] for the f32 instruction and D[4*v+l/16][l%16] for the f64 one.
template <typename T, int NG>
__global__ __launch_bounds__(256) void k_fit_gemm(const T* __restrict__ Q, const T* __restrict__ W,
                                                  T* __restrict__ gridlet, const int* __restrict__ leaves,
                                                  int first, int rows) {
  constexpr int M = NG * NG * NG, kpad = (M + 3) / 4 * 4, mpad = (M + 15) / 16 * 16;
  constexpr int CT = mpad / 16;       // column tiles
  constexpr int CH = (CT + 1) / 2;    // column tiles per wave
  constexpr int KC = kpad < 24 ? kpad : 24;  // K rows per LDS chunk (a multiple of 4)
  constexpr int KS = KC / 4;
  constexpr int MP2 = 2 * CH * 16;    // LDS row: both waves' tiles, zero past mpad
  using V4 = typename std::conditional<sizeof(T) == 4, floatx4, doublex4>::type;
  __shared__ T sW[KC * MP2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.x * 32 + (wave & 1) * 16;
  const int c0 = (wave >> 1) * CH;
  const int i = lane & 15, kk = lane >> 4;
  const int arow = row0 + i;
  const bool arow_ok = arow < rows;
  V4 acc[CH];
#pragma unroll
  for (int t = 0; t < CH; ++t) acc[t] = V4{T(0), T(0), T(0), T(0)};
  // W chunk rows k0 .. k0+KC into registers (all loads in flight together)
  constexpr int NF = (KC * MP2 + 255) / 256;
  T wreg[NF];
  auto load_w = [&](int k0) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int e = threadIdx.x + 256 * f;
      const int k = k0 + e / MP2, c = e % MP2;
      wreg[f] = (e < KC * MP2 && k < kpad && c < mpad) ? W[size_t(k) * mpad + c] : T(0);
    }
  };
  // the same chunk rows of this lane's Q row, likewise one chunk ahead
  T an[KS];
  auto load_a = [&](int k0) {
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int k = k0 + 4 * q + kk;
      an[q] = (arow_ok && k < kpad) ? Q[size_t(arow) * kpad + k] : T(0);
    }
  };
  load_w(0);
  load_a(0);
  for (int k0 = 0; k0 < kpad; k0 += KC) {
    T av[KS];
#pragma unroll
    for (int q = 0; q < KS; ++q) av[q] = an[q];
    __syncthreads();  // the previous chunk's reads are done
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int e = threadIdx.x + 256 * f;
      if (e < KC * MP2) sW[e] = wreg[f];
    }
    __syncthreads();
    if (k0 + KC < kpad) {  // next chunk in flight during this one's MFMAs
      load_w(k0 + KC);
      load_a(k0 + KC);
    }
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const T* wrow = sW + (4 * q + kk) * MP2 + c0 * 16 + i;
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const T bv = wrow[t * 16];
        if constexpr (sizeof(T) == 4) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], bv, acc[t], 0, 0, 0);
        else acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv, acc[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < CH; ++t) {
    const int c = (c0 + t) * 16 + i;
    if (c0 + t < CT && c < M) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + (sizeof(T) == 4 ? 4 * kk + v : 4 * v + kk);
        if (r < rows) gridlet[size_t(leaves[first + r]) * M + c] = acc[t][v];
      }
    }
  }
}

template <typename T, int NG>
__global__ __launch_bounds__(256) void k_m2m(int off, const int* __restrict__ flags,
                                             const int* __restrict__ child8, const T* __restrict__ t1,
                                             T* __restrict__ gridlet) {
  constexpr int M = NG * NG * NG;
  constexpr int PER = (M + 255) / 256;
  __shared__ T s_in[M], s_a[M], s_b[M];
  __shared__ T s_t[2][NG][NG];
  const int g = off + blockIdx.x;
  if (!(flags[g] & 1)) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * NG * NG; e += 256) (&s_t[0][0][0])[e] = t1[e];
  T out[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) out[r] = T(0);
  for (int c = 0; c < 8; ++c) {
    const int ch = child8[g * 8 + c];
    if (ch < 0) continue;
    const int ax = c & 1, ay = (c >> 1) & 1, az = (c >> 2) & 1;
    __syncthreads();
    for (int e = tid; e < M; e += 256) s_in[e] = gridlet[size_t(ch) * M + e];
    __syncthreads();
    for (int e = tid; e < M; e += 256) {
      const int px = e % NG, rest = e / NG;
      T acc = T(0);
#pragma unroll
      for (int q = 0; q < NG; ++q) acc += s_t[ax][px][q] * s_in[rest * NG + q];
      s_a[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < M; e += 256) {
      const int px = e % NG, py = (e / NG) % NG, qz = e / (NG * NG);
      T acc = T(0);
#pragma unroll
      for (int q = 0; q < NG; ++q) acc += s_t[ay][py][q] * s_a[(qz * NG + q) * NG + px];
      s_b[e] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 256 * r;
      if (e < M) {
        const int px = e % NG, py = (e / NG) % NG, pz = e / (NG * NG);
        T acc = T(0);
#pragma unroll
        for (int q = 0; q < NG; ++q) acc += s_t[az][pz][q] * s_b[(q * NG + py) * NG + px];
        out[r] += acc;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = tid + 256 * r;
    if (e < M) gridlet[size_t(g) * M + e] = out[r];
  }
}

static inline int nblk(int64_t n, int t) { return int((n + t - 1) / t); }

void launch_gather_masses(Plan& p, const void* m, hipStream_t s) {
  const int n = int(p.n);
  if (p.prec == HPM_F32)
    k_gather_masses<float><<<nblk(n, 256), 256, 0, s>>>(n, p.perm.as<int>(), (const float*)m, p.ms.as<float>());
  else
    k_gather_masses<double><<<nblk(n, 256), 256, 0, s>>>(n, p.perm.as<int>(), (const double*)m, p.ms.as<double>());
  HPM_LAUNCH_CHECK();
}

// moments and fit of `rows` cells listed in list[first ..]; levels from row_level or the ids
template <typename T, int NG>
static void p2m_rows(Plan& p, const int* list, int first, int rows, const int* row_level,
                     hipStream_t s) {
  if (rows <= 0) return;
  P2MArgs<T> a;
  a.leaves = list;
  a.row_level = row_level;
  a.first = first;
  a.count = rows;
  a.level_off = p.dlev.as<int>() + kLevOff;
  a.nlevels = p.nlevels;
  a.coord = p.ccoord.as<int>();
  a.pb = p.cpb.as<int>();
  a.pe = p.cpe.as<int>();
  a.xs = p.xs.as<T>();
  a.ys = p.ys.as<T>();
  a.zs = p.zs.as<T>();
  a.ms = p.ms.as<T>();
  a.moments = p.moments.as<T>();
  a.kpad = p.tab.kpad;
  a.lo0 = p.prob.box_lo[0];
  a.lo1 = p.prob.box_lo[1];
  a.lo2 = p.prob.box_lo[2];
  a.size = p.prob.box_size;
  k_p2m_moments<T, NG><<<rows, 64, 0, s>>>(a);
  HPM_LAUNCH_CHECK();
  k_fit_gemm<T, NG><<<nblk(rows, 32), 256, 0, s>>>(p.moments.as<T>(), p.tab.fitw.as<T>(), p.gridlet.as<T>(),
                                         list, first, rows);
  HPM_LAUNCH_CHECK();
}

// the leaves at levels >= 2 and the virtual cubes, in one pass over the combined row list
template <typename T, int NG>
static void p2m_t(Plan& p, hipStream_t s) {
  p2m_rows<T, NG>(p, p.p2m_list.as<int>(), 0, int(p.p2m_rows), p.p2m_level.as<int>(), s);
}

// rows of the fit: leaf r of levels >= 2 (list position first2 + r), then virtual cube v (cell
// id ncells + v), each with its level
__global__ void k_p2m_rows(int nl2, int first2, const int* leaves, int nvirt, int ncells,
                           const int* vlevel, const int* level_off, int nlevels, int* list,
                           int* level) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nl2) {
    const int g = leaves[first2 + r];
    list[r] = g;
    level[r] = level_of(g, level_off, nlevels);
  } else if (r < nl2 + nvirt) {
    list[r] = ncells + (r - nl2);
    level[r] = vlevel[r - nl2];
  }
}

void build_p2m_rows(Plan& p, hipStream_t s) {
  const int nl2 = int(p.nleaves - p.nleaves_lt2), nv = int(p.nvirt);
  p.p2m_rows = nl2 + nv;
  if (p.p2m_rows <= 0) return;
  p.p2m_list.reserve(size_t(p.p2m_rows) * 4);
  p.p2m_level.reserve(size_t(p.p2m_rows) * 4);
  k_p2m_rows<<<nblk(p.p2m_rows, 256), 256, 0, s>>>(nl2, int(p.nleaves_lt2), p.leaves.as<int>(), nv,
                                                   int(p.ncells), p.vlevel.as<int>(),
                                                   p.dlev.as<int>() + kLevOff, p.nlevels,
                                                   p.p2m_list.as<int>(), p.p2m_level.as<int>());
  HPM_LAUNCH_CHECK();
}

template <typename T, int NG>
static void m2m_t(Plan& p, int level, hipStream_t s) {
  const int off = p.level_off[level];
  const int cnt = p.level_off[level + 1] - off;
  if (cnt <= 0) return;
  k_m2m<T, NG><<<cnt, 256, 0, s>>>(off, p.cflags.as<int>(), p.child8.as<int>(), p.tab.m2m.as<T>(),
                                   p.gridlet.as<T>());
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

void launch_p2m(Plan& p, hipStream_t s) { HPM_DISPATCH_NG(p2m_t, p, s); }
void launch_m2m(Plan& p, int level, hipStream_t s) { HPM_DISPATCH_NG(m2m_t, p, level, s); }

}  // namespace hpm
