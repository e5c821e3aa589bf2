// Constant tables, built on the host in double precision and rounded once to the plan's dtype
// (the paper precomputes the Green function and the matrices A, B, T before timing, Sec. 4).
//
//   fit matrix   Effective masses from moments (Sec. 2.2, Eq. 4-5). The moments here are taken
//                in the tensor Legendre basis phi_n(x) = P_nx(2x) P_ny(2y) P_nz(2z), which spans
//                the same polynomials as the Cartesian monomials x^n of Eq. (2), so the matched
//                effective masses are identical; the fit matrix is B^phi = (Pmat)^{-1} with
//                Pmat[n][p] = phi_n(x_p), a Kronecker product of the 1-D inverse. Stored as the
//                GEMM operand W[n][p] = B^phi[p][n], zero padded.
//   child-to-parent  1-D factors of T^C (Sec. 2.3): T1^a[p][q] = l_p((a + x_q)/2) with
//                a = -1/2 or +1/2, the Lagrange basis l_p on the gridlet nodes (the matrix of
//                the paper's double sum, in closed form). Parent-to-child uses the transpose,
//                on the target gridlet's nodes (N_g + 2 of them when extended, Sec. 2.5).
//   Green transform  per level l >= 2: the exact lattice Green function G(d) = g(h_l |d|_p) of
//                Eq. (1) on the (8 N_g)^3 grid, h_l = size / (2^l N_g), with the problem's
//                kernel g (softened Newtonian -G (r^2+eps^2)^{-1/2}, or the screened one;
//                any kernel works, Sec. 4); for eps = 0 the origin takes the value at unit
//                offset. G is real and even along each axis, so its DFT is real, even and a
//                product of cosine sums; only the octant k in [0, n/2]^3 is stored, divided by
//                n^3 (the normalisation of the unnormalised inverse FFT). The same function
//                transformed along x and y only, at the z offsets 0 .. 4 N_g that separate a
//                target node from a source node (4 N_g = n/2 only with extended target gridlets),
//                and divided by n^2, serves the variant of the source-to-target step that
//                convolves along z in real space.
//   cell-by-cell Green transforms  (only for the cell-by-cell route, Sec. 2.5) per level and
//                source cube offset d in [-3, 3]^3: the C^3 cyclic array, C = 2 N_g + 2 ext,
//                whose entry u holds g(h_l |d N_g - u_c|), u_c = u for u < N_g + ext and u - C
//                otherwise, so that each node offset between a target node (N_g + 2 ext per
//                axis) and a source node sits on its own entry; its half spectrum
//                [kz][ky][kx <= C/2] by separable direct sums, divided by C^3, each offset's
//                row padded with zeros to a multiple of 16 modes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "hpm_internal.h"

namespace hpm {

// node i of a gridlet of N_g points per axis widened by ext nodes on each side
static double node(int ng, int i, int ext = 0) { return (2.0 * (i - ext) + 1.0 - ng) / (2.0 * ng); }

static double lagrange(int ng, int p, double u, int ext = 0) {
  double v = 1.0;
  for (int m = 0; m < ng + 2 * ext; ++m)
    if (m != p) v *= (u - node(ng, m, ext)) / (node(ng, p, ext) - node(ng, m, ext));
  return v;
}

static double legendre(int k, double t) {
  double p0 = 1.0, p1 = t;
  if (k == 0) return p0;
  for (int j = 1; j < k; ++j) {
    const double p2 = ((2.0 * j + 1.0) * t * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Gauss-Jordan inverse with partial pivoting of a small dense matrix (row-major, n x n).
static std::vector<double> invert(std::vector<double> a, int n) {
  std::vector<double> inv(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) inv[size_t(i) * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[size_t(r) * n + c]) > std::fabs(a[size_t(piv) * n + c])) piv = r;
    for (int k = 0; k < n; ++k) {
      std::swap(a[size_t(c) * n + k], a[size_t(piv) * n + k]);
      std::swap(inv[size_t(c) * n + k], inv[size_t(piv) * n + k]);
    }
    const double d = a[size_t(c) * n + c];
    for (int k = 0; k < n; ++k) {
      a[size_t(c) * n + k] /= d;
      inv[size_t(c) * n + k] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[size_t(r) * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[size_t(r) * n + k] -= f * a[size_t(c) * n + k];
        inv[size_t(r) * n + k] -= f * inv[size_t(c) * n + k];
      }
    }
  }
  return inv;
}

// Transforms of the cyclic Green arrays of the cell-by-cell route, all levels and offsets.
static std::vector<double> cell_green(const Plan& p, int nlev) {
  const int ng = p.ng, ext = p.ext, C = 2 * ng + 2 * ext, HC = C / 2 + 1;
  const int Kp = int(cell_modes(ng, ext));  // C^2 HC modes, padded
  std::vector<double> out(size_t(std::max(nlev, 1)) * 343 * Kp * 2, 0.0);
  std::vector<double> cs(size_t(C) * C), sn(size_t(C) * C);
  for (int k = 0; k < C; ++k)
    for (int j = 0; j < C; ++j) {
      const double ang = 2.0 * M_PI * double((k * j) % C) / double(C);
      cs[size_t(k) * C + j] = std::cos(ang);
      sn[size_t(k) * C + j] = -std::sin(ang);
    }
  const double G = p.prob.gconst, eps = p.prob.softening, inv = 1.0 / (double(C) * C * C);
  std::vector<double> g(size_t(C) * C * C);
  std::vector<double> a1r(size_t(C) * C * HC), a1i(a1r.size()), a2r(size_t(C) * C * HC),
      a2i(a2r.size());
  for (int li = 0; li < nlev; ++li) {
    const double h = p.prob.box_size / (double(1 << (li + 2)) * ng);
    for (int od = 0; od < 343; ++od) {
      const int d[3] = {od % 7 - 3, (od / 7) % 7 - 3, od / 49 - 3};
      if (std::abs(d[0]) <= 1 && std::abs(d[1]) <= 1 && std::abs(d[2]) <= 1) continue;  // near
      for (int z = 0; z < C; ++z)
        for (int y = 0; y < C; ++y)
          for (int x = 0; x < C; ++x) {
            const int u[3] = {x, y, z};
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
              const double o = double(d[a] * ng - (u[a] < ng + ext ? u[a] : u[a] - C));
              r2 += o * o;
            }
            const double sd = std::sqrt(r2 * h * h + eps * eps);
            g[(size_t(z) * C + y) * C + x] = (p.prob.kernel == HPM_KERNEL_YUKAWA)
                                                 ? -G * std::exp(-sd / p.prob.screening) / sd
                                                 : -G / sd;
          }
      // x (real input): a1[z][y][kx]
      for (int zy = 0; zy < C * C; ++zy)
        for (int kx = 0; kx < HC; ++kx) {
          double re = 0.0, im = 0.0;
          for (int x = 0; x < C; ++x) {
            re += g[size_t(zy) * C + x] * cs[size_t(kx) * C + x];
            im += g[size_t(zy) * C + x] * sn[size_t(kx) * C + x];
          }
          a1r[size_t(zy) * HC + kx] = re;
          a1i[size_t(zy) * HC + kx] = im;
        }
      // y: a2[z][ky][kx]
      for (int z = 0; z < C; ++z)
        for (int ky = 0; ky < C; ++ky)
          for (int kx = 0; kx < HC; ++kx) {
            double re = 0.0, im = 0.0;
            for (int y = 0; y < C; ++y) {
              const size_t i = (size_t(z) * C + y) * HC + kx;
              const double c = cs[size_t(ky) * C + y], sv = sn[size_t(ky) * C + y];
              re += a1r[i] * c - a1i[i] * sv;
              im += a1r[i] * sv + a1i[i] * c;
            }
            a2r[(size_t(z) * C + ky) * HC + kx] = re;
            a2i[(size_t(z) * C + ky) * HC + kx] = im;
          }
      // z: [kz][ky][kx], interleaved (re, im), / C^3
      double* o = &out[(size_t(li) * 343 + od) * Kp * 2];
      for (int kz = 0; kz < C; ++kz)
        for (int col = 0; col < C * HC; ++col) {
          double re = 0.0, im = 0.0;
          for (int z = 0; z < C; ++z) {
            const size_t i = size_t(z) * C * HC + col;
            const double c = cs[size_t(kz) * C + z], sv = sn[size_t(kz) * C + z];
            re += a2r[i] * c - a2i[i] * sv;
            im += a2r[i] * sv + a2i[i] * c;
          }
          o[(size_t(kz) * C * HC + col) * 2] = re * inv;
          o[(size_t(kz) * C * HC + col) * 2 + 1] = im * inv;
        }
    }
  }
  return out;
}

template <typename T>
static void upload(DevBuf& buf, const std::vector<double>& v, hipStream_t s) {
  std::vector<T> h(v.begin(), v.end());
  buf.reserve(h.size() * sizeof(T));
  HPM_HIP(hipMemcpyAsync(buf.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  HPM_HIP(hipStreamSynchronize(s));
}

void build_tables(Plan& p, int max_levels, hipStream_t s) {
  const int ng = p.ng, M = ng * ng * ng;
  // 1-D Legendre-at-nodes matrix and its inverse
  std::vector<double> pm(size_t(ng) * ng);
  for (int k = 0; k < ng; ++k)
    for (int q = 0; q < ng; ++q) pm[size_t(k) * ng + q] = legendre(k, 2.0 * node(ng, q));
  const std::vector<double> b1 = invert(pm, ng);  // b1[p][k]
  const int kpad = (M + 3) / 4 * 4, mpad = (M + 15) / 16 * 16;
  std::vector<double> w(size_t(kpad) * mpad, 0.0);
  for (int nz = 0; nz < ng; ++nz)
    for (int ny = 0; ny < ng; ++ny)
      for (int nx = 0; nx < ng; ++nx)
        for (int pz = 0; pz < ng; ++pz)
          for (int py = 0; py < ng; ++py)
            for (int px = 0; px < ng; ++px) {
              const int n = nx + ng * (ny + ng * nz), q = px + ng * (py + ng * pz);
              w[size_t(n) * mpad + q] = b1[size_t(px) * ng + nx] * b1[size_t(py) * ng + ny] *
                                        b1[size_t(pz) * ng + nz];
            }
  p.tab.kpad = kpad;
  p.tab.mpad = mpad;

  std::vector<double> t1(size_t(2) * ng * ng);
  for (int a = 0; a < 2; ++a)
    for (int pp = 0; pp < ng; ++pp)
      for (int q = 0; q < ng; ++q)
        t1[(size_t(a) * ng + pp) * ng + q] = lagrange(ng, pp, ((a ? 0.5 : -0.5) + node(ng, q)) / 2.0);
  const int nl = p.NL;
  std::vector<double> t1l(size_t(2) * nl * nl);
  for (int a = 0; a < 2; ++a)
    for (int pp = 0; pp < nl; ++pp)
      for (int q = 0; q < nl; ++q)
        t1l[(size_t(a) * nl + pp) * nl + q] =
            lagrange(ng, pp, ((a ? 0.5 : -0.5) + node(ng, q, p.ext)) / 2.0, p.ext);

  // Green transforms, levels 2 .. nlevels-1
  const int n = 8 * ng, H = n / 2 + 1;
  const int nlev = std::max(0, max_levels - 2);
  std::vector<double> ghat(size_t(std::max(nlev, 1)) * H * H * H, 0.0);
  const int D = 4 * ng + 1;
  std::vector<double> gxy(size_t(std::max(nlev, 1)) * D * H * H, 0.0);
  std::vector<double> cs(size_t(H) * n);
  for (int k = 0; k < H; ++k)
    for (int d = 0; d < n; ++d)
      cs[size_t(k) * n + d] = std::cos(2.0 * M_PI * double((long(k) * d) % n) / double(n));
  std::vector<int> pd(n);
  for (int i = 0; i < n; ++i) pd[i] = (i <= n / 2) ? i : n - i;
  const double G = p.prob.gconst, eps = p.prob.softening;
  std::vector<double> g(size_t(n) * n * n), a1(size_t(n) * n * H), a2(size_t(n) * H * H);
  for (int li = 0; li < nlev; ++li) {
    const int l = li + 2;
    const double h = p.prob.box_size / (double(1 << l) * ng);
    for (int z = 0; z < n; ++z)
      for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
          double r2 = h * h * double(pd[x] * pd[x] + pd[y] * pd[y] + pd[z] * pd[z]);
          if (x == 0 && y == 0 && z == 0 && eps == 0.0) r2 = h * h;
          // Offsets with max-norm <= N_g join a target node only to nodes of the 27 cubes
          // around the target, which are not sources; every interaction-zone pair is at least
          // N_g + 1 apart along some axis (N_g with the extended target gridlet, whose outer
          // nodes lie one spacing closer to the sources). Their values never reach a target
          // potential, and zero keeps the largest (near-origin) kernel values out of the
          // transform, where they would only add rounding error.
          const bool unreachable = std::max(pd[x], std::max(pd[y], pd[z])) <= ng - p.ext;
          double gv = 0.0;
          if (!unreachable) {
            const double sd = std::sqrt(r2 + eps * eps);
            gv = (p.prob.kernel == HPM_KERNEL_YUKAWA) ? -G * std::exp(-sd / p.prob.screening) / sd
                                                      : -G / sd;
          }
          g[(size_t(z) * n + y) * n + x] = gv;
        }
    // x: a1[z][y][kx]
    for (int z = 0; z < n; ++z)
      for (int y = 0; y < n; ++y)
        for (int kx = 0; kx < H; ++kx) {
          double acc = 0.0;
          const double* row = &g[(size_t(z) * n + y) * n];
          for (int x = 0; x < n; ++x) acc += row[x] * cs[size_t(kx) * n + x];
          a1[(size_t(z) * n + y) * H + kx] = acc;
        }
    // y: a2[z][ky][kx]
    for (int z = 0; z < n; ++z)
      for (int ky = 0; ky < H; ++ky)
        for (int kx = 0; kx < H; ++kx) {
          double acc = 0.0;
          for (int y = 0; y < n; ++y) acc += a1[(size_t(z) * n + y) * H + kx] * cs[size_t(ky) * n + y];
          a2[(size_t(z) * H + ky) * H + kx] = acc;
        }
    // x, y only: gxy[d][ky][kx] = a2[d][ky][kx] / n^2, d <= 4 N_g
    const double inv_n2 = 1.0 / (double(n) * n);
    for (size_t e = 0; e < size_t(D) * H * H; ++e) gxy[size_t(li) * D * H * H + e] = a2[e] * inv_n2;
    // z: ghat[kz][ky][kx] / n^3
    const double inv_n3 = 1.0 / (double(n) * n * n);
    double* out = &ghat[size_t(li) * H * H * H];
    for (int kz = 0; kz < H; ++kz)
      for (int ky = 0; ky < H; ++ky)
        for (int kx = 0; kx < H; ++kx) {
          double acc = 0.0;
          for (int z = 0; z < n; ++z) acc += a2[(size_t(z) * H + ky) * H + kx] * cs[size_t(kz) * n + z];
          out[(size_t(kz) * H + ky) * H + kx] = acc * inv_n3;
        }
  }
  p.tab.ghat_levels = nlev;
  if (p.prob.m2l_mode != HPM_M2L_GRID) {
    const std::vector<double> gc = cell_green(p, nlev);
    if (p.prec == HPM_F32) upload<float>(p.tab.gcell, gc, s);
    else upload<double>(p.tab.gcell, gc, s);
    p.tab.gcell_levels = nlev;
  }
  if (p.prec == HPM_F32) {
    // e^{+2 pi i m / n} as float pairs (hi, lo) per component, for the all-FP32 inverse
    // transform: {cos hi, sin hi, cos lo, sin lo}
    const int nn = 8 * p.ng;
    std::vector<double> tw(size_t(nn) * 4);
    for (int m = 0; m < nn; ++m) {
      const double c = std::cos(2.0 * M_PI * m / nn), sn = std::sin(2.0 * M_PI * m / nn);
      const float ch = float(c), sh = float(sn);
      tw[4 * m] = ch;
      tw[4 * m + 1] = sh;
      tw[4 * m + 2] = float(c - double(ch));
      tw[4 * m + 3] = float(sn - double(sh));
    }
    upload<float>(p.tab.twff, tw, s);
    upload<float>(p.tab.fitw, w, s);
    upload<float>(p.tab.m2m, t1, s);
    upload<float>(p.tab.l2l, t1l, s);
    upload<float>(p.tab.ghat, ghat, s);
    upload<float>(p.tab.gxy, gxy, s);
  } else {
    upload<double>(p.tab.fitw, w, s);
    upload<double>(p.tab.m2m, t1, s);
    upload<double>(p.tab.l2l, t1l, s);
    upload<double>(p.tab.ghat, ghat, s);
    upload<double>(p.tab.gxy, gxy, s);
  }
}

}  // namespace hpm
