// kernels.hpp -- HIP kernels (gfx950) of one hybrid lattice Boltzmann
// timestep: the stencil force fused with the forced BGK collide-and-stream
// (Sec. 2.1 and 2.2 of the paper), and the finite-difference
// convection-diffusion substep (Sec. 2.3).
//
// Device data layout (structure of arrays, 256-byte aligned):
//   g[i*ns + idx]  population deviations g_i = f_i - w_i rho0, stored
//                  post-collision and pre-streaming, so that one step reads
//                  every population once with a pull (g_i from r - e_i) and
//                  writes it once, coalesced, at r.  The pre-collision value
//                  at time t at site r is therefore g_i(r - e_i).
//   phi[idx]       order parameter at time t.
//   u[k*ns + idx]  u* of the last step (input of the convection-diffusion
//                  substeps).
// idx = x + nx*(y + ny*z).  Every kernel works on a tile of TX x TY (x TZ)
// sites; the stencil inputs of a tile, with their halo, are staged in LDS
// once and every derived stencil quantity (lap phi or mu, the advected h,
// the diffusion potential) is computed once per tile site in LDS, so each
// value is read from HBM once and each stencil is evaluated once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace hlb {

// Parameters of a launch, in double; kernels convert to their storage type.
struct KParams {
  int nx, ny, nz, ns;
  double a, b, kappa;
  double omega;          // 1 / tau
  double gamma;          // mobility
  double gN, gM;         // gradient stencil (Eq. xstencil): axis and transverse weights
  double lQ, lR, lC;     // force Laplacian (Eq. laplstencil): face, edge, centre
  double cQ, cR, cC;     // Laplacian of the convection-diffusion step
  double dt;             // Delta t_FD = 1/m
  double g[3];           // body acceleration
  double rho0;
  int force_form;        // 1 expanded, 0 mu-first
  int advection;         // 0 paper, 1 flux form
};

__device__ __forceinline__ int wrapc(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// ---------------------------------------------------------------- stencils
// Laplacian of Eq. laplstencil on an LDS tile at (x, y, z): weight Q on the
// axis neighbours, R on the diagonal (edge) neighbours, C at the centre.
template <int D, typename T, int PX, int PY, int PZ>
__device__ __forceinline__ T lap_at(const T (&s)[PZ][PY][PX], int x, int y, int z, T Q, T R, T C) {
  if constexpr (D == 2) {
    const T faces = (s[0][y][x + 1] + s[0][y][x - 1]) + (s[0][y + 1][x] + s[0][y - 1][x]);
    const T edges = (s[0][y + 1][x + 1] + s[0][y + 1][x - 1]) + (s[0][y - 1][x + 1] + s[0][y - 1][x - 1]);
    return Q * faces + R * edges + C * s[0][y][x];
  } else {
    const T faces = (s[z][y][x + 1] + s[z][y][x - 1]) + (s[z][y + 1][x] + s[z][y - 1][x]) +
                    (s[z + 1][y][x] + s[z - 1][y][x]);
    const T exy = (s[z][y + 1][x + 1] + s[z][y + 1][x - 1]) + (s[z][y - 1][x + 1] + s[z][y - 1][x - 1]);
    const T exz = (s[z + 1][y][x + 1] + s[z + 1][y][x - 1]) + (s[z - 1][y][x + 1] + s[z - 1][y][x - 1]);
    const T eyz = (s[z + 1][y + 1][x] + s[z + 1][y - 1][x]) + (s[z - 1][y + 1][x] + s[z - 1][y - 1][x]);
    return Q * faces + R * (exy + exz + eyz) + C * s[z][y][x];
  }
}

// Gradient of Eq. xstencil: weight N on the axis neighbours, M on the edge
// neighbours that have one transverse offset; y (and z) by transposition.
template <int D, typename T, int PX, int PY, int PZ>
__device__ __forceinline__ void grad_at(const T (&s)[PZ][PY][PX], int x, int y, int z, T N, T M, T g[3]) {
  if constexpr (D == 2) {
    g[0] = N * (s[0][y][x + 1] - s[0][y][x - 1]) +
           M * ((s[0][y + 1][x + 1] - s[0][y + 1][x - 1]) + (s[0][y - 1][x + 1] - s[0][y - 1][x - 1]));
    g[1] = N * (s[0][y + 1][x] - s[0][y - 1][x]) +
           M * ((s[0][y + 1][x + 1] - s[0][y - 1][x + 1]) + (s[0][y + 1][x - 1] - s[0][y - 1][x - 1]));
    g[2] = T(0);
  } else {
    g[0] = N * (s[z][y][x + 1] - s[z][y][x - 1]) +
           M * ((s[z][y + 1][x + 1] - s[z][y + 1][x - 1]) + (s[z][y - 1][x + 1] - s[z][y - 1][x - 1]) +
                (s[z + 1][y][x + 1] - s[z + 1][y][x - 1]) + (s[z - 1][y][x + 1] - s[z - 1][y][x - 1]));
    g[1] = N * (s[z][y + 1][x] - s[z][y - 1][x]) +
           M * ((s[z][y + 1][x + 1] - s[z][y - 1][x + 1]) + (s[z][y + 1][x - 1] - s[z][y - 1][x - 1]) +
                (s[z + 1][y + 1][x] - s[z + 1][y - 1][x]) + (s[z - 1][y + 1][x] - s[z - 1][y - 1][x]));
    g[2] = N * (s[z + 1][y][x] - s[z - 1][y][x]) +
           M * ((s[z + 1][y][x + 1] - s[z - 1][y][x + 1]) + (s[z + 1][y][x - 1] - s[z - 1][y][x - 1]) +
                (s[z + 1][y + 1][x] - s[z - 1][y + 1][x]) + (s[z + 1][y - 1][x] - s[z - 1][y - 1][x]));
  }
}

// Stage field[] over the box starting at global (gx0, gy0, gz0) (periodic
// wrap) into an LDS tile.
template <int D, typename T, int PX, int PY, int PZ>
__device__ __forceinline__ void load_tile(T (&s)[PZ][PY][PX], const T *__restrict__ field, const KParams &p,
                                          int gx0, int gy0, int gz0) {
  for (int i = threadIdx.x; i < PX * PY * PZ; i += blockDim.x) {
    const int lx = i % PX, ly = (i / PX) % PY, lz = i / (PX * PY);
    const int gx = wrapc(gx0 + lx, p.nx), gy = wrapc(gy0 + ly, p.ny);
    const int gz = (D == 3) ? wrapc(gz0 + lz, p.nz) : 0;
    s[lz][ly][lx] = field[gx + p.nx * (gy + p.ny * gz)];
  }
}

// ------------------------------------------------------------ force tile
// The force needs phi with a halo of 2 and lap_D phi (or mu) with a halo of
// 1 around the tile.
template <int D, typename T, int TX, int TY, int TZ>
struct ForceTile {
  static constexpr int H = 2;
  static constexpr int PX = TX + 4, PY = TY + 4, PZ = D == 3 ? TZ + 4 : 1;
  static constexpr int LX = TX + 2, LY = TY + 2, LZ = D == 3 ? TZ + 2 : 1;
  T phi[PZ][PY][PX];
  T lam[LZ][LY][LX];  // lap_D phi (expanded form) or mu (mu-first form)

  __device__ __forceinline__ void build(const T *__restrict__ gphi, const KParams &p, int x0, int y0, int z0) {
    load_tile<D>(phi, gphi, p, x0 - H, y0 - H, D == 3 ? z0 - H : 0);
    __syncthreads();
    const T Q = T(p.lQ), R = T(p.lR), C = T(p.lC);
    const T a = T(p.a), b = T(p.b), kappa = T(p.kappa);
    const bool mu_first = p.force_form == 0;
    for (int i = threadIdx.x; i < LX * LY * LZ; i += blockDim.x) {
      const int lx = i % LX, ly = (i / LX) % LY, lz = i / (LX * LY);
      const int px = lx + 1, py = ly + 1, pz = D == 3 ? lz + 1 : 0;
      const T l = lap_at<D>(phi, px, py, pz, Q, R, C);
      if (mu_first) {
        const T ph = phi[pz][py][px];
        lam[lz][ly][lx] = a * ph + b * ph * ph * ph - kappa * l;
      } else {
        lam[lz][ly][lx] = l;
      }
    }
    __syncthreads();
  }

  // Force density at tile site (tx, ty, tz), without the body-force term;
  // also returns phi and mu there.
  __device__ __forceinline__ void force(const KParams &p, int tx, int ty, int tz, T F[3], T &ph, T &mu) const {
    const int px = tx + H, py = ty + H, pz = D == 3 ? tz + H : 0;
    const int lx = tx + 1, ly = ty + 1, lz = D == 3 ? tz + 1 : 0;
    const T N = T(p.gN), M = T(p.gM);
    const T a = T(p.a), b = T(p.b), kappa = T(p.kappa);
    ph = phi[pz][py][px];
    T gl[3];
    grad_at<D>(lam, lx, ly, lz, N, M, gl);
    if (p.force_form == 0) {
      mu = lam[lz][ly][lx];
#pragma unroll
      for (int k = 0; k < 3; k++) F[k] = -ph * gl[k];
    } else {
      T gp[3];
      grad_at<D>(phi, px, py, pz, N, M, gp);
      const T ph3 = ph * ph * ph;
      mu = a * ph + b * ph3 - kappa * lam[lz][ly][lx];
      const T bulk = a * ph + T(3) * b * ph3;
#pragma unroll
      for (int k = 0; k < 3; k++) F[k] = -(bulk * gp[k] - kappa * ph * gl[k]);
    }
  }
};

// Pull the pre-collision populations of site (x, y, z) (g_i from r - e_i,
// periodic) and form the moments: dn = sum g_i (n = rho0 + dn), j = sum g_i e_i.
template <class L, typename T>
__device__ __forceinline__ void pull(const KParams &p, const T *__restrict__ g, int x, int y, int z, T f[L::Q],
                                     T &dn, T j[3]) {
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int xs[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
  const int ys[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
  const int zs[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
  dn = T(0);
  j[0] = j[1] = j[2] = T(0);
  const size_t ns = (size_t)p.ns;
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    const int ex = L::e(i, 0), ey = L::e(i, 1), ez = L::e(i, 2);
    int src;
    if constexpr (L::D == 2)
      src = xs[1 - ex] + nx * ys[1 - ey];
    else
      src = xs[1 - ex] + nx * (ys[1 - ey] + ny * zs[1 - ez]);
    f[i] = g[(size_t)i * ns + src];
  }
  // sums in a fixed order, independent of the load schedule
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    dn += f[i];
    if (L::e(i, 0) == 1) j[0] += f[i];
    if (L::e(i, 0) == -1) j[0] -= f[i];
    if (L::e(i, 1) == 1) j[1] += f[i];
    if (L::e(i, 1) == -1) j[1] -= f[i];
    if (L::D == 3 && L::e(i, 2) == 1) j[2] += f[i];
    if (L::D == 3 && L::e(i, 2) == -1) j[2] -= f[i];
  }
}

// ------------------------------------------------------------------ kernels
// Force (Eq. forza) + moments (Eq. newvel) + forced BGK collision
// (Eqs. espdistrfunc, forceevoleqn, latticeforceterm) + streaming.
// Writes the post-collision populations of time t at r (pull storage) and u*_t.
template <class L, typename T, int TX, int TY, int TZ>
__global__ void __launch_bounds__(256) k_lb(KParams p, const T *__restrict__ gin, T *__restrict__ gout,
                                            const T *__restrict__ phi, T *__restrict__ uout) {
  constexpr int D = L::D;
  __shared__ ForceTile<D, T, TX, TY, TZ> tile;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = D == 3 ? blockIdx.z * TZ : 0;
  tile.build(phi, p, x0, y0, z0);

  const T rho0 = T(p.rho0), omega = T(p.omega);
  const T fac = T(1) - T(0.5) * omega;  // 1 - 1/(2 tau)
  const size_t ns = (size_t)p.ns;
  for (int s = threadIdx.x; s < TX * TY * TZ; s += blockDim.x) {
    const int tx = s % TX, ty = (s / TX) % TY, tz = s / (TX * TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    if (x >= p.nx || y >= p.ny || z >= p.nz) continue;
    const int idx = x + p.nx * (y + p.ny * z);

    T F[3], ph, mu;
    tile.force(p, tx, ty, tz, F, ph, mu);
    T f[L::Q], dn, j[3];
    pull<L>(p, gin, x, y, z, f, dn, j);
    const T n = rho0 + dn;
    T u[3];
    const T inv_n = T(1) / n;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      F[k] += n * T(p.g[k]);
      u[k] = (j[k] + T(0.5) * F[k]) * inv_n;
    }
#pragma unroll
    for (int k = 0; k < D; k++) uout[k * ns + idx] = u[k];

    const T usq = u[0] * u[0] + u[1] * u[1] + (D == 3 ? u[2] * u[2] : T(0));
    const T uF = u[0] * F[0] + u[1] * F[1] + (D == 3 ? u[2] * F[2] : T(0));
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
      const int ex = L::e(i, 0), ey = L::e(i, 1), ez = L::e(i, 2);
      const T eu = T(ex) * u[0] + T(ey) * u[1] + (D == 3 ? T(ez) * u[2] : T(0));
      const T eF = T(ex) * F[0] + T(ey) * F[1] + (D == 3 ? T(ez) * F[2] : T(0));
      const T w = T(L::w(i));
      // g^eq = f^eq - w rho0 = w [dn + n (3 e.u + 9/2 (e.u)^2 - 3/2 u.u)]
      const T geq = w * (dn + n * (T(3) * eu + T(4.5) * eu * eu - T(1.5) * usq));
      // lattice forcing term, (1 - 1/2tau) w [3 (e - u).F + 9 (e.u)(e.F)]
      const T S = fac * w * (T(3) * (eF - uF) + T(9) * eu * eF);
      gout[(size_t)i * ns + idx] = f[i] - omega * (f[i] - geq) + S;
    }
  }
}

// One convection-diffusion substep (Sec. 2.3): advection half-step
// h = phi - dt [phi div_c u + u . D^up phi] (Eqs. adv, centrdiff, backdiff,
// fordiff; or the flux form), then phi' = h + dt Gamma L[a h + b phi^3 - kappa L h],
// which equals Eq. diff, h + dt Gamma [a L h + b L phi^3 - kappa L L h], by
// linearity of L.
template <class L, typename T, int TX, int TY, int TZ>
__global__ void __launch_bounds__(256) k_ch(KParams p, const T *__restrict__ phi_in, const T *__restrict__ u,
                                            T *__restrict__ phi_out) {
  constexpr int D = L::D;
  constexpr int H = 3;
  constexpr int PX = TX + 6, PY = TY + 6, PZ = D == 3 ? TZ + 6 : 1;
  constexpr int HX = TX + 4, HY = TY + 4, HZ = D == 3 ? TZ + 4 : 1;
  constexpr int MX = TX + 2, MY = TY + 2, MZ = D == 3 ? TZ + 2 : 1;
  __shared__ T sphi[PZ][PY][PX];
  __shared__ T sh[HZ][HY][HX];
  __shared__ T smu[MZ][MY][MX];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = D == 3 ? blockIdx.z * TZ : 0;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const size_t ns = (size_t)p.ns;
  load_tile<D>(sphi, phi_in, p, x0 - H, y0 - H, D == 3 ? z0 - H : 0);
  __syncthreads();

  const T dt = T(p.dt);
  const bool flux = p.advection == 1;
  // advection half-step on the tile plus a halo of 2
  for (int i = threadIdx.x; i < HX * HY * HZ; i += blockDim.x) {
    const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
    const int px = hx + 1, py = hy + 1, pz = D == 3 ? hz + 1 : 0;
    const int gx = wrapc(x0 - 2 + hx, nx), gy = wrapc(y0 - 2 + hy, ny);
    const int gz = D == 3 ? wrapc(z0 - 2 + hz, nz) : 0;
    const int gxm = gx == 0 ? nx - 1 : gx - 1, gxp = gx == nx - 1 ? 0 : gx + 1;
    const int gym = gy == 0 ? ny - 1 : gy - 1, gyp = gy == ny - 1 ? 0 : gy + 1;
    const int gzm = gz == 0 ? nz - 1 : gz - 1, gzp = gz == nz - 1 ? 0 : gz + 1;
    const int c = gx + nx * (gy + ny * gz);
    const T ph = sphi[pz][py][px];
    T rhs = T(0);
#pragma unroll
    for (int a = 0; a < D; a++) {
      int im, ip;
      T pm, pp;
      if (a == 0) {
        im = gxm + nx * (gy + ny * gz);
        ip = gxp + nx * (gy + ny * gz);
        pm = sphi[pz][py][px - 1];
        pp = sphi[pz][py][px + 1];
      } else if (a == 1) {
        im = gx + nx * (gym + ny * gz);
        ip = gx + nx * (gyp + ny * gz);
        pm = sphi[pz][py - 1][px];
        pp = sphi[pz][py + 1][px];
      } else {
        im = gx + nx * (gy + ny * gzm);
        ip = gx + nx * (gy + ny * gzp);
        pm = sphi[pz - 1][py][px];
        pp = sphi[pz + 1][py][px];
      }
      const T *ua = u + a * ns;
      const T uc = ua[c], um = ua[im], up = ua[ip];
      if (!flux) {
        const T dcu = (up - um) * T(0.5);
        const T dup = uc > T(0) ? ph - pm : pp - ph;
        rhs += ph * dcu + uc * dup;
      } else {
        const T vp = (uc + up) * T(0.5), vm = (um + uc) * T(0.5);
        const T Pp = vp > T(0) ? vp * ph : vp * pp;
        const T Pm = vm > T(0) ? vm * pm : vm * ph;
        rhs += Pp - Pm;
      }
    }
    sh[hz][hy][hx] = ph - dt * rhs;
  }
  __syncthreads();

  const T a = T(p.a), b = T(p.b), kappa = T(p.kappa);
  const T cQ = T(p.cQ), cR = T(p.cR), cC = T(p.cC);
  // diffusion potential a h + b phi^3 - kappa L h on the tile plus a halo of 1
  for (int i = threadIdx.x; i < MX * MY * MZ; i += blockDim.x) {
    const int mx = i % MX, my = (i / MX) % MY, mz = i / (MX * MY);
    const int hx = mx + 1, hy = my + 1, hz = D == 3 ? mz + 1 : 0;
    const int px = mx + 2, py = my + 2, pz = D == 3 ? mz + 2 : 0;
    const T ph = sphi[pz][py][px];
    const T h = sh[hz][hy][hx];
    smu[mz][my][mx] = a * h + b * ph * ph * ph - kappa * lap_at<D>(sh, hx, hy, hz, cQ, cR, cC);
  }
  __syncthreads();

  const T dtg = dt * T(p.gamma);
  for (int s = threadIdx.x; s < TX * TY * TZ; s += blockDim.x) {
    const int tx = s % TX, ty = (s / TX) % TY, tz = s / (TX * TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    if (x >= nx || y >= ny || z >= nz) continue;
    const int mx = tx + 1, my = ty + 1, mz = D == 3 ? tz + 1 : 0;
    const int hx = tx + 2, hy = ty + 2, hz = D == 3 ? tz + 2 : 0;
    phi_out[x + nx * (y + ny * z)] = sh[hz][hy][hx] + dtg * lap_at<D>(smu, mx, my, mz, cQ, cR, cC);
  }
}

// f_i = f_i^eq(n0, u0) (Eq. espdistrfunc) from double-precision inputs
// io = [phi | n | u (d components)]; stored pull-wise, g_i(r) = f_i(r + e_i) - w_i rho0.
template <class L, typename T>
__global__ void __launch_bounds__(256) k_init(KParams p, const double *__restrict__ io, T *__restrict__ gout,
                                              T *__restrict__ phi) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= p.ns) return;
  const size_t ns = (size_t)p.ns;
  const int x = idx % p.nx, y = (idx / p.nx) % p.ny, z = idx / (p.nx * p.ny);
  const double *n0 = io + ns, *u0 = io + 2 * ns;
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    const int sx = wrapc(x + L::e(i, 0), p.nx), sy = wrapc(y + L::e(i, 1), p.ny);
    const int sz = L::D == 3 ? wrapc(z + L::e(i, 2), p.nz) : 0;
    const int src = sx + p.nx * (sy + p.ny * sz);
    const double n = n0[src];
    double eu = 0.0, usq = 0.0;
    for (int k = 0; k < L::D; k++) {
      const double uk = u0[k * ns + src];
      eu += L::e(i, k) * uk;
      usq += uk * uk;
    }
    const double w = L::w(i);
    const double geq = w * ((n - p.rho0) + n * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
    gout[(size_t)i * ns + idx] = T(geq);
  }
  phi[idx] = T(io[idx]);
}

// Raw state I/O, one population at a time (runtime velocity (ex, ey, ez)).
// get: out[r] = f_i(r) = g_i(r - e_i) + w_i rho0.
template <typename T>
__global__ void __launch_bounds__(256) k_get_pop(KParams p, const T *__restrict__ gi, int ex, int ey, int ez,
                                                 double w, double *__restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= p.ns) return;
  const int x = idx % p.nx, y = (idx / p.nx) % p.ny, z = idx / (p.nx * p.ny);
  const int src = wrapc(x - ex, p.nx) + p.nx * (wrapc(y - ey, p.ny) + p.ny * wrapc(z - ez, p.nz));
  out[idx] = double(gi[src]) + w * p.rho0;
}

// set: g_i(r) = f_i(r + e_i) - w_i rho0.
template <typename T>
__global__ void __launch_bounds__(256) k_set_pop(KParams p, const double *__restrict__ in, int ex, int ey, int ez,
                                                 double w, T *__restrict__ gi) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= p.ns) return;
  const int x = idx % p.nx, y = (idx / p.nx) % p.ny, z = idx / (p.nx * p.ny);
  const int src = wrapc(x + ex, p.nx) + p.nx * (wrapc(y + ey, p.ny) + p.ny * wrapc(z + ez, p.nz));
  gi[idx] = T(in[src] - w * p.rho0);
}

template <typename T>
__global__ void __launch_bounds__(256) k_convert(int n, const double *__restrict__ in, T *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = T(in[i]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_widen(int n, const T *__restrict__ in, double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = double(in[i]);
}

// Fields at time t into io = [n | u* (d) | phi | mu], double precision.
template <class L, typename T, int TX, int TY, int TZ>
__global__ void __launch_bounds__(256) k_readout(KParams p, const T *__restrict__ gin, const T *__restrict__ phi,
                                                 double *__restrict__ io) {
  constexpr int D = L::D;
  __shared__ ForceTile<D, T, TX, TY, TZ> tile;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = D == 3 ? blockIdx.z * TZ : 0;
  tile.build(phi, p, x0, y0, z0);
  const size_t ns = (size_t)p.ns;
  for (int s = threadIdx.x; s < TX * TY * TZ; s += blockDim.x) {
    const int tx = s % TX, ty = (s / TX) % TY, tz = s / (TX * TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    if (x >= p.nx || y >= p.ny || z >= p.nz) continue;
    const int idx = x + p.nx * (y + p.ny * z);
    T F[3], ph, mu;
    tile.force(p, tx, ty, tz, F, ph, mu);
    T f[L::Q], dn, j[3];
    pull<L>(p, gin, x, y, z, f, dn, j);
    const T n = T(p.rho0) + dn;
    const T inv_n = T(1) / n;
    io[idx] = double(n);
#pragma unroll
    for (int k = 0; k < D; k++) {
      const T Fk = F[k] + n * T(p.g[k]);
      io[(1 + k) * ns + idx] = double((j[k] + T(0.5) * Fk) * inv_n);
    }
    io[(1 + D) * ns + idx] = double(ph);
    io[(2 + D) * ns + idx] = double(mu);
  }
}

// Global diagnostics, stage 1: per-block partial sums in double.
// part[blk*8 + k]: 0 mass, 1 phi, 2 kinetic, 3..5 momentum, 6 max|u*|, 7 non-finite count.
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}

// Block reduction of 8 values in a fixed order (blockDim = 256 = 4 waves).
__device__ __forceinline__ void block_reduce8(double v[8], double *out) {
  __shared__ double red[4][8];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 8; k++) v[k] = (k == 6) ? wave_max(v[k]) : wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 8; k++) red[wid][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 8; k++) {
      double r = red[0][k];
      for (int w = 1; w < 4; w++) r = (k == 6) ? fmax(r, red[w][k]) : r + red[w][k];
      out[k] = r;
    }
  }
}

template <class L, typename T, int TX, int TY, int TZ>
__global__ void __launch_bounds__(256) k_reduce(KParams p, const T *__restrict__ gin, const T *__restrict__ phi,
                                                double *__restrict__ part) {
  constexpr int D = L::D;
  __shared__ ForceTile<D, T, TX, TY, TZ> tile;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = D == 3 ? blockIdx.z * TZ : 0;
  tile.build(phi, p, x0, y0, z0);
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = threadIdx.x; s < TX * TY * TZ; s += blockDim.x) {
    const int tx = s % TX, ty = (s / TX) % TY, tz = s / (TX * TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    if (x >= p.nx || y >= p.ny || z >= p.nz) continue;
    T F[3], ph, mu;
    tile.force(p, tx, ty, tz, F, ph, mu);
    T f[L::Q], dn, j[3];
    pull<L>(p, gin, x, y, z, f, dn, j);
    bool finite = isfinite(double(ph));
#pragma unroll
    for (int i = 0; i < L::Q; i++) finite = finite && isfinite(double(f[i]));
    const T n = T(p.rho0) + dn;
    const T inv_n = T(1) / n;
    double u2 = 0.0;
    double nd = double(n);
#pragma unroll
    for (int k = 0; k < D; k++) {
      const T Fk = F[k] + n * T(p.g[k]);
      const double uk = double((j[k] + T(0.5) * Fk) * inv_n);
      u2 += uk * uk;
      acc[3 + k] += nd * uk;
    }
    acc[0] += nd;
    acc[1] += double(ph);
    acc[2] += 0.5 * nd * u2;
    acc[6] = fmax(acc[6], sqrt(u2));
    acc[7] += finite ? 0.0 : 1.0;
  }
  const int blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  block_reduce8(acc, part + (size_t)blk * 8);
}

// Stage 2: one block folds the partials in a fixed order.
__global__ void __launch_bounds__(256) k_reduce_final(int nblk, const double *__restrict__ part,
                                                      double *__restrict__ out) {
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < 8; k++) acc[k] = (k == 6) ? fmax(acc[k], part[(size_t)b * 8 + k]) : acc[k] + part[(size_t)b * 8 + k];
  block_reduce8(acc, out);
}

}  // namespace hlb
