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

#include <utility>

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
  double omega_h;        // D2Q5 convection-diffusion model: 1 / tau_phi
  double gamma_h;        // and Gamma / (tau_phi - 1/2)
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
// wrap) into an LDS tile.  When the lattice is at least as large as the box
// on every axis a single conditional wrap is exact; smaller lattices (tiles
// that wrap more than once) take the modulo path.  The branch is uniform.
__device__ __forceinline__ int wrap1(int v, int n) {
  v += v < 0 ? n : 0;
  return v >= n ? v - n : v;
}

// Upwind terms of the advection half-step (Sec. 2.3) without a branch.
// Written as a select between two neighbour values, the compiler moves each
// neighbour's LDS load into its own divergent branch and waits for it there,
// which serialises two LDS latencies per term; selecting on the velocity
// instead issues both loads together.  For finite values the results equal
// the selected forms up to the order of rounding in a fused multiply-add.
// u (c - m) where u > 0, else u (p - c)  (one-sided difference upwind of u)
template <typename T>
__device__ __forceinline__ T upwind_diff(T u, T m, T c, T p) {
  const bool pos = u > T(0);
  return (pos ? u : T(0)) * (c - m) + (pos ? T(0) : u) * (p - c);
}
// v l where v > 0, else v r  (face flux of the upwind cell value)
template <typename T>
__device__ __forceinline__ T upwind_flux(T v, T l, T r) {
  const bool pos = v > T(0);
  return (pos ? v : T(0)) * l + (pos ? T(0) : v) * r;
}

// Threads per block of every stencil kernel.
constexpr int NT = 256;

// Global -> LDS staging in two halves: issue() puts all of a thread's loads
// in flight into registers, commit() writes them to LDS.  Issuing every load
// of a kernel (tiles and populations) before the first use keeps the memory
// pipeline full instead of paying one latency per loop iteration.
// Block coordinates with an XCD-aware order.  The hardware hands workgroup i
// (linear id, x fastest) to XCD i mod 8; remapping so that each XCD owns a
// contiguous range of tiles keeps neighbouring tiles, whose halos overlap,
// in the same L2.
__device__ __forceinline__ void tile_coords(int &bx, int &by, int &bz) {
  constexpr int NXCD = 8;
  const int gx = gridDim.x, gy = gridDim.y;
  const int nblk = gx * gy * gridDim.z;
  const int bid = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int q = nblk / NXCD, r = nblk % NXCD;
  const int xcd = bid % NXCD, pos = bid / NXCD;
  const int lid = xcd * q + min(xcd, r) + pos;
  bx = lid % gx;
  by = (lid / gx) % gy;
  bz = lid / (gx * gy);
}

template <int D, typename T, int PX, int PY, int PZ, int NTH = NT>
struct TileLoad {
  static constexpr int N = PX * PY * PZ;
  static constexpr int K = (N + NTH - 1) / NTH;
  T v[K];

  __device__ __forceinline__ void issue(const T *__restrict__ field, const KParams &p, int gx0, int gy0, int gz0) {
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const bool inside = gx0 >= 0 && gx0 + PX <= nx && gy0 >= 0 && gy0 + PY <= ny &&
                        (D == 2 || (gz0 >= 0 && gz0 + PZ <= nz));
    if (inside) {  // no periodic image involved
      const T *base = field + gx0 + nx * (gy0 + ny * (D == 3 ? gz0 : 0));
#pragma unroll
      for (int k = 0; k < K; k++) {
        const int i = threadIdx.x + k * NTH;
        if (N % NTH == 0 || i < N) {
          const int lx = i % PX, ly = (i / PX) % PY, lz = i / (PX * PY);
          v[k] = base[lx + nx * (ly + ny * lz)];
        }
      }
      return;
    }
    const bool fast = nx >= PX && ny >= PY && (D == 2 || nz >= PZ);
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      if (N % NTH == 0 || i < N) {
        const int lx = i % PX, ly = (i / PX) % PY, lz = i / (PX * PY);
        int gx, gy, gz = 0;
        if (fast) {
          gx = wrap1(gx0 + lx, nx);
          gy = wrap1(gy0 + ly, ny);
          if (D == 3) gz = wrap1(gz0 + lz, nz);
        } else {
          gx = wrapc(gx0 + lx, nx);
          gy = wrapc(gy0 + ly, ny);
          if (D == 3) gz = wrapc(gz0 + lz, nz);
        }
        v[k] = field[gx + nx * (gy + ny * gz)];
      }
    }
  }

  // Writes the tile into a 2D LDS array with row pitch PITCH, element (x, y)
  // at s[y * PITCH + OFFX + x].
  template <int PITCH, int OFFX>
  __device__ __forceinline__ void commit_pitched(T *s) const {
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      if (N % NTH == 0 || i < N) s[(i / PX) * PITCH + OFFX + i % PX] = v[k];
    }
  }

  __device__ __forceinline__ void commit(T (&s)[PZ][PY][PX]) const {
    T *flat = &s[0][0][0];
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      if (N % NTH == 0 || i < N) flat[i] = v[k];
    }
  }
};

template <int D, typename T, int PX, int PY, int PZ>
__device__ __forceinline__ void load_tile(T (&s)[PZ][PY][PX], const T *__restrict__ field, const KParams &p,
                                          int gx0, int gy0, int gz0) {
  TileLoad<D, T, PX, PY, PZ> t;
  t.issue(field, p, gx0, gy0, gz0);
  t.commit(s);
}

// Laplacian with R = 0 (the standard 5/7-point operator): axis neighbours only.
template <int D, typename T, int PX, int PY, int PZ>
__device__ __forceinline__ T lap5_at(const T (&s)[PZ][PY][PX], int x, int y, int z, T Q, T C) {
  if constexpr (D == 2) {
    return Q * ((s[0][y][x + 1] + s[0][y][x - 1]) + (s[0][y + 1][x] + s[0][y - 1][x])) + C * s[0][y][x];
  } else {
    return Q * ((s[z][y][x + 1] + s[z][y][x - 1]) + (s[z][y + 1][x] + s[z][y - 1][x]) +
                (s[z + 1][y][x] + s[z - 1][y][x])) +
           C * s[z][y][x];
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

  using Loader = TileLoad<D, T, PX, PY, PZ>;

  __device__ __forceinline__ void issue(Loader &ld, const T *__restrict__ gphi, const KParams &p, int x0, int y0,
                                        int z0) const {
    ld.issue(gphi, p, x0 - H, y0 - H, D == 3 ? z0 - H : 0);
  }

  // Commit phi to LDS and form lap_D phi (or mu) on the tile plus a halo of 1.
  __device__ __forceinline__ void finish(const Loader &ld, const KParams &p) {
    ld.commit(phi);
    __syncthreads();
    const T Q = T(p.lQ), R = T(p.lR), C = T(p.lC);
    const T a = T(p.a), b = T(p.b), kappa = T(p.kappa);
    const bool mu_first = p.force_form == 0;
    for (int i = threadIdx.x; i < LX * LY * LZ; i += NT) {
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

  __device__ __forceinline__ void build(const T *__restrict__ gphi, const KParams &p, int x0, int y0, int z0) {
    Loader ld;
    issue(ld, gphi, p, x0, y0, z0);
    finish(ld, p);
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

// Pull the pre-collision populations of site (x, y, z): g_i from r - e_i
// (periodic).  Loads only; moments() forms the sums.
template <class L, typename T>
__device__ __forceinline__ void pull_issue(const KParams &p, const T *__restrict__ g, int x, int y, int z,
                                           T f[L::Q]) {
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int xs[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
  const int ys[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
  const int zs[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
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
}

// dn = sum g_i (n = rho0 + dn) and j = sum g_i e_i, in a fixed order.
template <class L, typename T>
__device__ __forceinline__ void moments(const T f[L::Q], T &dn, T j[3]) {
  dn = T(0);
  j[0] = j[1] = j[2] = T(0);
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

template <class L, typename T>
__device__ __forceinline__ void pull(const KParams &p, const T *__restrict__ g, int x, int y, int z, T f[L::Q],
                                     T &dn, T j[3]) {
  pull_issue<L>(p, g, x, y, z, f);
  moments<L>(f, dn, j);
}

// Forced BGK collision of one site, written to the post-collision store.
// With f^eq of Eq. espdistrfunc at u* and the forcing term of
// Eq. latticeforceterm, post_i = (1 - w) f_i + w f_i^eq + F_i (w = 1/tau)
// splits, for a velocity and its opposite, into a part even in e_i and a
// part odd in e_i:
//   post_{+-} = (1 - omega) g_{+-} + w_i [A + eu (B eu + C eF)] +- w_i [D eu + E eF]
// with eu = e_i.u*, eF = e_i.F and the site constants
//   A = omega (dn - 3/2 n u.u) - 3 (1 - omega/2) u.F,  B = 9/2 omega n,
//   C = 9 (1 - omega/2),  D = 3 omega n,  E = 3 (1 - omega/2),
// so each pair costs one evaluation.  Populations are deviations
// g = f - w rho0 (dn = n - rho0).
template <class L, typename T>
__device__ __forceinline__ void collide(const T f[L::Q], T dn, T n, const T u[3], const T F[3], T omega, T fac,
                                        T *__restrict__ gout, size_t ns, int idx) {
  constexpr int D = L::D;
  const T usq = u[0] * u[0] + u[1] * u[1] + (D == 3 ? u[2] * u[2] : T(0));
  const T uF = u[0] * F[0] + u[1] * F[1] + (D == 3 ? u[2] * F[2] : T(0));
  const T om1 = T(1) - omega;
  const T A = omega * (dn - T(1.5) * n * usq) - T(3) * fac * uF;
  const T B = T(4.5) * omega * n, C = T(9) * fac, Dc = T(3) * omega * n, E = T(3) * fac;
  gout[idx] = om1 * f[0] + T(L::w(0)) * A;
#pragma unroll
  for (int i = 1; i < L::Q; i++) {
    const int o = L::opp(i);
    if (o < i) continue;
    const int ex = L::e(i, 0), ey = L::e(i, 1), ez = L::e(i, 2);
    const T eu = T(ex) * u[0] + T(ey) * u[1] + (D == 3 ? T(ez) * u[2] : T(0));
    const T eF = T(ex) * F[0] + T(ey) * F[1] + (D == 3 ? T(ez) * F[2] : T(0));
    const T w = T(L::w(i));
    const T sym = w * (A + eu * (B * eu + C * eF));
    const T asym = w * (Dc * eu + E * eF);
    gout[(size_t)i * ns + idx] = om1 * f[i] + (sym + asym);
    gout[(size_t)o * ns + idx] = om1 * f[o] + (sym - asym);
  }
}

// ------------------------------------------------------------------ kernels
// Force (Eq. forza) + moments (Eq. newvel) + forced BGK collision
// (Eqs. espdistrfunc, forceevoleqn, latticeforceterm) + streaming.
// Writes the post-collision populations of time t at r (pull storage) and u*_t.
// With CD5 (D2Q9 only), the D2Q5 lattice Boltzmann alternative for the
// convection-diffusion equation runs in the same pass: its populations h_i
// (stored like g, post-collision at the site of origin, velocities the first
// five of D2Q9) are pulled, relaxed with omega_h towards
//   h_i^eq = w_i (Gamma_h mu + phi c_i.u*) / c_s^2 (i = 1..4),
//   h_0^eq = phi - sum_{i>0} h_i^eq,
// with mu = a phi + b phi^3 - kappa L phi (the convection-diffusion
// Laplacian, from the staged phi tile), and stored to hout; u* is not
// stored.  phi of the next step is the sum of the pulled h (k_phi5).
template <class L, typename T, int TX, int TY, int TZ, bool CD5 = false>
__device__ __forceinline__ void lb_tile(const KParams &p, const T *__restrict__ gin, T *__restrict__ gout,
                                        const T *__restrict__ phi, T *__restrict__ uout, int x0, int y0, int z0,
                                        const T *__restrict__ hin = nullptr, T *__restrict__ hout = nullptr) {
  constexpr int D = L::D;
  constexpr int NSITE = (TX * TY * TZ + NT - 1) / NT;  // sites per thread
  static_assert(!CD5 || D == 2, "the D2Q5 model is two-dimensional");
  using FT = ForceTile<D, T, TX, TY, TZ>;
  __shared__ FT tile;

  // all global loads first: this thread's populations, then the phi tile
  T f[NSITE][L::Q];
  T h[NSITE][5];
  int sx[NSITE], sy[NSITE], sz[NSITE];
  bool ok[NSITE];
#pragma unroll
  for (int k = 0; k < NSITE; k++) {
    const int s = threadIdx.x + k * NT;
    const int tx = s % TX, ty = (s / TX) % TY, tz = s / (TX * TY);
    sx[k] = tx;
    sy[k] = ty;
    sz[k] = tz;
    ok[k] = s < TX * TY * TZ && x0 + tx < p.nx && y0 + ty < p.ny && z0 + tz < p.nz;
    if (ok[k]) pull_issue<L>(p, gin, x0 + tx, y0 + ty, z0 + tz, f[k]);
    if constexpr (CD5) {
      if (ok[k]) {
        const int x = x0 + tx, y = y0 + ty, nx = p.nx, ny = p.ny;
        const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
        const size_t ns = (size_t)p.ns;
        h[k][0] = hin[x + nx * y];
        h[k][1] = hin[ns + xm + nx * y];      // c_1 = (+1, 0): from x - 1
        h[k][2] = hin[2 * ns + x + nx * ym];  // c_2 = (0, +1): from y - 1
        h[k][3] = hin[3 * ns + xp + nx * y];  // c_3 = (-1, 0): from x + 1
        h[k][4] = hin[4 * ns + x + nx * yp];  // c_4 = (0, -1): from y + 1
      }
    }
  }
  typename FT::Loader ld;
  tile.issue(ld, phi, p, x0, y0, z0);
  tile.finish(ld, p);

  const T rho0 = T(p.rho0), omega = T(p.omega);
  const T fac = T(1) - T(0.5) * omega;  // 1 - 1/(2 tau)
  const size_t ns = (size_t)p.ns;
#pragma unroll
  for (int k = 0; k < NSITE; k++) {
    if (!ok[k]) continue;
    const int tx = sx[k], ty = sy[k], tz = sz[k];
    const int idx = (x0 + tx) + p.nx * ((y0 + ty) + p.ny * (z0 + tz));
    T F[3], ph, mu;
    tile.force(p, tx, ty, tz, F, ph, mu);
    T dn, j[3];
    moments<L>(f[k], dn, j);
    const T n = rho0 + dn;
    T u[3];
    const T inv_n = T(1) / n;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      F[c] += n * T(p.g[c]);
      u[c] = (j[c] + T(0.5) * F[c]) * inv_n;
    }
    if constexpr (!CD5) {
#pragma unroll
      for (int c = 0; c < D; c++) uout[c * ns + idx] = u[c];
    } else {
      const int px = tx + FT::H, py = ty + FT::H;
      T lap;
      if (p.cR == 0.0)
        lap = lap5_at<2>(tile.phi, px, py, 0, T(p.cQ), T(p.cC));
      else
        lap = lap_at<2>(tile.phi, px, py, 0, T(p.cQ), T(p.cR), T(p.cC));
      const T mu5 = T(p.a) * ph + T(p.b) * ph * ph * ph - T(p.kappa) * lap;
      const T A = T(0.5) * T(p.gamma_h) * mu5;  // w_i Gamma_h mu / c_s^2, w_i = 1/6
      const T bx = T(0.5) * ph * u[0], by = T(0.5) * ph * u[1];
      const T om = T(p.omega_h);
      const T eq[5] = {ph - T(4) * A, A + bx, A + by, A - bx, A - by};
#pragma unroll
      for (int i = 0; i < 5; i++) hout[(size_t)i * ns + idx] = h[k][i] + om * (eq[i] - h[k][i]);
    }

    collide<L>(f[k], dn, n, u, F, omega, fac, gout, ns, idx);
  }
}

template <class L, typename T, int TX, int TY, int TZ>
__global__ void __launch_bounds__(NT) k_lb(KParams p, const T *__restrict__ gin, T *__restrict__ gout,
                                           const T *__restrict__ phi, T *__restrict__ uout) {
  int bx, by, bz;
  tile_coords(bx, by, bz);
  lb_tile<L, T, TX, TY, TZ>(p, gin, gout, phi, uout, bx * TX, by * TY, L::D == 3 ? bz * TZ : 0);
}

// The D2Q9 step with the D2Q5 convection-diffusion model (see lb_tile).
template <typename T, int TX, int TY>
__global__ void __launch_bounds__(NT) k_lb5(KParams p, const T *__restrict__ gin, T *__restrict__ gout,
                                            const T *__restrict__ phi, const T *__restrict__ hin,
                                            T *__restrict__ hout) {
  int bx, by, bz;
  tile_coords(bx, by, bz);
  lb_tile<D2Q9, T, TX, TY, 1, true>(p, gin, gout, phi, nullptr, bx * TX, by * TY, 0, hin, hout);
}

// phi(r) = sum_i h_i(r) of the D2Q5 model, with the pre-collision h_i(r)
// pulled from the stores at r - c_i, summed in the order i = 0..4.
template <typename T>
__global__ void __launch_bounds__(256) k_phi5(KParams p, const T *__restrict__ h, T *__restrict__ phi) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= p.ns) return;
  const int nx = p.nx, ny = p.ny, x = idx % nx, y = idx / nx;
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const size_t ns = (size_t)p.ns;
  T s = h[idx];
  s += h[ns + xm + nx * y];
  s += h[2 * ns + x + nx * ym];
  s += h[3 * ns + xp + nx * y];
  s += h[4 * ns + x + nx * yp];
  phi[idx] = s;
}

// Initial D2Q5 populations h_i = h_i^eq(phi0, mu0, u0) from double-precision
// io = [phi | n | u_x | u_y], stored pull-wise: store_i(r) = h_i(r + c_i).
template <typename T>
__global__ void __launch_bounds__(256) k_init5(KParams p, const double *__restrict__ io, T *__restrict__ h) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= p.ns) return;
  const int nx = p.nx, ny = p.ny, x = idx % nx, y = idx / nx;
  const size_t ns = (size_t)p.ns;
  const int cx[5] = {0, 1, 0, -1, 0}, cy[5] = {0, 0, 1, 0, -1};
#pragma unroll
  for (int i = 0; i < 5; i++) {
    const int sx = wrapc(x + cx[i], nx), sy = wrapc(y + cy[i], ny);
    auto at = [&](int dx, int dy) { return io[wrapc(sx + dx, nx) + nx * wrapc(sy + dy, ny)]; };
    const double ph = at(0, 0);
    const double faces = (at(1, 0) + at(-1, 0)) + (at(0, 1) + at(0, -1));
    const double edges = (at(1, 1) + at(-1, 1)) + (at(1, -1) + at(-1, -1));
    const double lap = p.cQ * faces + p.cR * edges + p.cC * ph;
    const double mu = p.a * ph + p.b * ph * ph * ph - p.kappa * lap;
    const double A = 0.5 * p.gamma_h * mu;
    const int src = sx + nx * sy;
    const double ux = io[2 * ns + src], uy = io[3 * ns + src];
    const double e[5] = {ph - 4.0 * A, A + 0.5 * ph * ux, A + 0.5 * ph * uy, A - 0.5 * ph * ux, A - 0.5 * ph * uy};
    h[(size_t)i * ns + idx] = T(e[i]);
  }
}

// One convection-diffusion substep (Sec. 2.3): advection half-step
// h = phi - dt [phi div_c u + u . D^up phi] (Eqs. adv, centrdiff, backdiff,
// fordiff; or the flux form), then phi' = h + dt Gamma L[a h + b phi^3 - kappa L h],
// which equals Eq. diff, h + dt Gamma [a L h + b L phi^3 - kappa L L h], by
// linearity of L.  phi and u* are staged with a halo of 3, h is formed on the
// tile plus a halo of 2 and the diffusion potential on the tile plus 1, all
// in LDS.  LAP5: the Laplacian has no edge weights (cd_Q = 1).
template <class L, typename T, int TX, int TY, int TZ, bool LAP5>
__device__ __forceinline__ void ch_tile(const KParams &p, const T *__restrict__ phi_in, const T *__restrict__ u,
                                        T *__restrict__ phi_out, int x0, int y0, int z0) {
  constexpr int D = L::D;
  constexpr int H = 3;
  constexpr int PX = TX + 6, PY = TY + 6, PZ = D == 3 ? TZ + 6 : 1;
  constexpr int HX = TX + 4, HY = TY + 4, HZ = D == 3 ? TZ + 4 : 1;
  constexpr int MX = TX + 2, MY = TY + 2, MZ = D == 3 ? TZ + 2 : 1;
  __shared__ T sphi[PZ][PY][PX];
  __shared__ T su[D][PZ][PY][PX];
  __shared__ T sh[HZ][HY][HX];
  __shared__ T smu[MZ][MY][MX];
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const size_t ns = (size_t)p.ns;
  {
    TileLoad<D, T, PX, PY, PZ> lphi, lu[D];
    lphi.issue(phi_in, p, x0 - H, y0 - H, D == 3 ? z0 - H : 0);
#pragma unroll
    for (int a = 0; a < D; a++) lu[a].issue(u + a * ns, p, x0 - H, y0 - H, D == 3 ? z0 - H : 0);
    lphi.commit(sphi);
#pragma unroll
    for (int a = 0; a < D; a++) lu[a].commit(su[a]);
  }
  __syncthreads();

  const T dt = T(p.dt);
  const bool flux = p.advection == 1;
  // advection half-step on the tile plus a halo of 2
  for (int i = threadIdx.x; i < HX * HY * HZ; i += NT) {
    const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
    const int px = hx + 1, py = hy + 1, pz = D == 3 ? hz + 1 : 0;
    const T ph = sphi[pz][py][px];
    T rhs = T(0);
#pragma unroll
    for (int a = 0; a < D; a++) {
      const int ox = a == 0, oy = a == 1, oz = a == 2;
      const T pm = sphi[pz - oz][py - oy][px - ox], pp = sphi[pz + oz][py + oy][px + ox];
      const T um = su[a][pz - oz][py - oy][px - ox], uc = su[a][pz][py][px], up = su[a][pz + oz][py + oy][px + ox];
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
  for (int i = threadIdx.x; i < MX * MY * MZ; i += NT) {
    const int mx = i % MX, my = (i / MX) % MY, mz = i / (MX * MY);
    const int hx = mx + 1, hy = my + 1, hz = D == 3 ? mz + 1 : 0;
    const int px = mx + 2, py = my + 2, pz = D == 3 ? mz + 2 : 0;
    const T ph = sphi[pz][py][px];
    const T h = sh[hz][hy][hx];
    const T Lh = LAP5 ? lap5_at<D>(sh, hx, hy, hz, cQ, cC) : lap_at<D>(sh, hx, hy, hz, cQ, cR, cC);
    smu[mz][my][mx] = a * h + b * ph * ph * ph - kappa * Lh;
  }
  __syncthreads();

  const T dtg = dt * T(p.gamma);
  for (int s = threadIdx.x; s < TX * TY * TZ; s += blockDim.x) {
    const int tx = s % TX, ty = (s / TX) % TY, tz = s / (TX * TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    if (x >= nx || y >= ny || z >= nz) continue;
    const int mx = tx + 1, my = ty + 1, mz = D == 3 ? tz + 1 : 0;
    const int hx = tx + 2, hy = ty + 2, hz = D == 3 ? tz + 2 : 0;
    const T Lmu = LAP5 ? lap5_at<D>(smu, mx, my, mz, cQ, cC) : lap_at<D>(smu, mx, my, mz, cQ, cR, cC);
    phi_out[x + nx * (y + ny * z)] = sh[hz][hy][hx] + dtg * Lmu;
  }
}

template <class L, typename T, int TX, int TY, int TZ, bool LAP5>
__global__ void __launch_bounds__(NT) k_ch(KParams p, const T *__restrict__ phi_in, const T *__restrict__ u,
                                            T *__restrict__ phi_out) {
  int bx, by, bz;
  tile_coords(bx, by, bz);
  ch_tile<L, T, TX, TY, TZ, LAP5>(p, phi_in, u, phi_out, bx * TX, by * TY, L::D == 3 ? bz * TZ : 0);
}

// ------------------------------------------------------- batched simulations
// Many independent periodic D2Q9 simulations of different sizes and
// parameters advanced together: one launch covers the tiles of every
// simulation, each block looking up its tile and its simulation.
struct SimDesc {
  KParams p;            // lattice size, coefficients and dt = 1/m of this simulation
  long long g[2];       // element offsets of the two population buffers
  long long phi[2];     // element offsets of the two phi buffers
  long long u;          // element offset of u*
  int m;                // convection-diffusion substeps per step
  int nl;               // substep launches per step that touch this simulation
  int phibase;          // phi buffer at the start of an even step
  int pad;
};

struct TileRef {
  int sim, x0, y0, pad;
};

// Batched simulations share one step parity `par` (steps since the start,
// mod 2): populations are read from buffer par and written to 1 - par.  Each
// substep launch that touches a simulation flips its phi buffer, nl times a
// step, so a simulation's phi starts a step in buffer phibase ^ (par & nl & 1).
__device__ __forceinline__ int batch_phi_buf(const SimDesc &sd, int par) { return sd.phibase ^ (par & sd.nl & 1); }

template <typename T, int TX, int TY>
__global__ void __launch_bounds__(NT) k_lb_batch(const SimDesc *__restrict__ sims, const TileRef *__restrict__ tiles,
                                                 T *__restrict__ g, T *__restrict__ phi, T *__restrict__ u, int par) {
  int b, unused1, unused2;
  tile_coords(b, unused1, unused2);
  const TileRef tr = tiles[b];
  const SimDesc &sd = sims[tr.sim];  // read in place: a private copy would live in scratch
  lb_tile<D2Q9, T, TX, TY, 1>(sd.p, g + sd.g[par], g + sd.g[1 - par], phi + sd.phi[batch_phi_buf(sd, par)],
                              u + sd.u, tr.x0, tr.y0, 0);
}

// Substep j of every simulation with m > j (one substep per launch).  The
// substep tile table lists the simulations in decreasing m, so the launch
// covers a prefix of it and every block has work.  Launch j reads phi from
// buffer (start ^ jpar) and writes the other; jpar = j & 1 in a step (a
// timing run passes 0: it then reads the state and writes the spare buffer).
template <typename T, int TX, int TY, bool LAP5>
__global__ void __launch_bounds__(NT) k_ch_batch(const SimDesc *__restrict__ sims, const TileRef *__restrict__ tiles,
                                                 T *__restrict__ phi, const T *__restrict__ u, int par, int j,
                                                 int jpar, int, int) {
  int b, unused1, unused2;
  tile_coords(b, unused1, unused2);
  const TileRef tr = tiles[b];
  const SimDesc &sd = sims[tr.sim];
  const int src = batch_phi_buf(sd, par) ^ jpar;
  ch_tile<D2Q9, T, TX, TY, 1, LAP5>(sd.p, phi + sd.phi[src], u + sd.u, phi + sd.phi[1 - src], tr.x0, tr.y0, 0);
}

// Substeps jM .. min((j+1)M, m) - 1 of every simulation with m > jM in one
// launch, on TO x TO tiles (2D): phi and u* are staged once with a halo of
// 3M and each substep works on a region that shrinks by 3 on every side
// (advection 1 + the two Laplacians of Eq. diff), entirely in LDS, as one
// substep does: h with a halo of 2, the diffusion potential with a halo of
// 1, then phi^{s+1} written over phi^s.  A simulation whose last launch has
// fewer than M substeps left stops early (its output region is then wider
// than needed).  Per launch phi and u* are read once and phi' written once.
template <typename T, int M, int TO, bool LAP5>
__global__ void __launch_bounds__(NT) k_chf_batch(const SimDesc *__restrict__ sims, const TileRef *__restrict__ tiles,
                                                  T *__restrict__ phi, const T *__restrict__ u, int par, int j,
                                                  int jpar, int, int) {
  constexpr int H = 3 * M;
  constexpr int L0 = TO + 2 * H;  // staged region edge
  __shared__ T sphi[1][L0][L0], sux[1][L0][L0], suy[1][L0][L0];
  __shared__ T sh[1][L0 - 2][L0 - 2], smu[1][L0 - 4][L0 - 4];
  int b, unused1, unused2;
  tile_coords(b, unused1, unused2);
  const TileRef tr = tiles[b];
  const SimDesc &sd = sims[tr.sim];
  const KParams &p = sd.p;
  const int src = batch_phi_buf(sd, par) ^ jpar;
  const T *__restrict__ phi_in = phi + sd.phi[src];
  T *__restrict__ phi_out = phi + sd.phi[1 - src];
  const T *__restrict__ us = u + sd.u;
  const int nsub = min(M, sd.m - j * M);
  const int x0 = tr.x0, y0 = tr.y0;
  const size_t ns = (size_t)p.ns;
  {
    TileLoad<2, T, L0, L0, 1> lphi, lux, luy;
    lphi.issue(phi_in, p, x0 - H, y0 - H, 0);
    lux.issue(us, p, x0 - H, y0 - H, 0);
    luy.issue(us + ns, p, x0 - H, y0 - H, 0);
    lphi.commit(sphi);
    lux.commit(sux);
    luy.commit(suy);
  }
  __syncthreads();
  const T dt = T(p.dt), dtg = T(p.dt) * T(p.gamma);
  const T a = T(p.a), bb = T(p.b), kappa = T(p.kappa), cQ = T(p.cQ), cR = T(p.cR), cC = T(p.cC);
  const bool flux = p.advection == 1;

  for (int s = 0; s < nsub; s++) {
    // input region of substep s: [3s, L0 - 3s) on both axes of the staged box
    const int lo = 3 * s;
    const int LH = L0 - 6 * s - 2;  // h region edge, origin lo + 1
    for (int i = threadIdx.x; i < LH * LH; i += NT) {
      const int y = lo + 1 + i / LH, x = lo + 1 + i % LH;
      const T pc = sphi[0][y][x];
      const T pw = sphi[0][y][x - 1], pe = sphi[0][y][x + 1];
      const T pdn = sphi[0][y - 1][x], pup = sphi[0][y + 1][x];
      const T uxc = sux[0][y][x], uxw = sux[0][y][x - 1], uxe = sux[0][y][x + 1];
      const T uyc = suy[0][y][x], uyd = suy[0][y - 1][x], uyu = suy[0][y + 1][x];
      T rhs;
      if (!flux) {
        const T tx = pc * ((uxe - uxw) * T(0.5)) + uxc * (uxc > T(0) ? pc - pw : pe - pc);
        const T ty = pc * ((uyu - uyd) * T(0.5)) + uyc * (uyc > T(0) ? pc - pdn : pup - pc);
        rhs = tx + ty;
      } else {
        const T vxe = (uxc + uxe) * T(0.5), vxw = (uxw + uxc) * T(0.5);
        const T vyu = (uyc + uyu) * T(0.5), vyd = (uyd + uyc) * T(0.5);
        const T tx = (vxe > T(0) ? vxe * pc : vxe * pe) - (vxw > T(0) ? vxw * pw : vxw * pc);
        const T ty = (vyu > T(0) ? vyu * pc : vyu * pup) - (vyd > T(0) ? vyd * pdn : vyd * pc);
        rhs = tx + ty;
      }
      sh[0][y - 1][x - 1] = pc - dt * rhs;
    }
    __syncthreads();
    const int LM = LH - 2;  // potential region edge, origin lo + 2
    for (int i = threadIdx.x; i < LM * LM; i += NT) {
      const int y = lo + 2 + i / LM, x = lo + 2 + i % LM;
      const int hy = y - 1, hx = x - 1;
      const T hc = sh[0][hy][hx];
      const T Lh = LAP5 ? lap5_at<2>(sh, hx, hy, 0, cQ, cC) : lap_at<2>(sh, hx, hy, 0, cQ, cR, cC);
      const T ph = sphi[0][y][x];
      smu[0][y - 2][x - 2] = a * hc + bb * ph * ph * ph - kappa * Lh;
    }
    __syncthreads();
    const int LO = LM - 2;  // output region edge, origin lo + 3
    for (int i = threadIdx.x; i < LO * LO; i += NT) {
      const int y = lo + 3 + i / LO, x = lo + 3 + i % LO;
      const int my = y - 2, mx = x - 2;
      const T Lm = LAP5 ? lap5_at<2>(smu, mx, my, 0, cQ, cC) : lap_at<2>(smu, mx, my, 0, cQ, cR, cC);
      sphi[0][y][x] = sh[0][y - 1][x - 1] + dtg * Lm;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < TO * TO; i += NT) {
    const int ty = i / TO, tx = i % TO;
    const int x = x0 + tx, y = y0 + ty;
    if (x < p.nx && y < p.ny) phi_out[x + p.nx * y] = sphi[0][H + ty][H + tx];
  }
}

// M convection-diffusion substeps in one pass (2D, standard 5-point
// Laplacian).  A block of BW threads owns BW consecutive lattice columns
// (one per thread) and marches along y.  One substep of Sec. 2.3 reads phi
// three rows away (advection 1 + the two Laplacians of Eq. diff), so the
// output row of substep s trails its newest input row by 3; substep s+1
// takes that row as input one iteration later, so every substep of an
// iteration works on values of the previous iteration and the M substeps
// are independent instruction streams (substep s runs 4s rows behind the
// input).  Each thread keeps, per substep, the last rows of phi^s, h and the
// diffusion potential of its column in registers (the y neighbours); the x
// neighbours come from one LDS row per quantity that every thread publishes
// at the start of an iteration, and u* from an LDS ring of its last 4M rows.
// One barrier per row.  Output columns: the middle BW - 6M; output rows: the
// segment [y0, y1) of the block.  phi and u* are read once and phi' written
// once per site for all M substeps.
// The block's output columns are [X0, X0 + ncol) (ncol <= BW - 6M) and its
// output rows [y0, y1).
template <typename T, int M, int BW>
struct MarchLds {
  T xphi[2][M][BW], xh[2][M][BW], xmu[2][M][BW];
  T sux[4 * M][BW], suy[4 * M][BW];
};

template <typename T, int M, int BW, bool FLUX>
__device__ __forceinline__ void ch_march_body(MarchLds<T, M, BW> &lds, const KParams &p, int X0, int ncol, int y0,
                                              int y1, const T *__restrict__ phi_in, const T *__restrict__ u,
                                              T *__restrict__ phi_out) {
  constexpr int R = 4 * M;  // rows of the u* ring
  auto &xphi = lds.xphi, &xh = lds.xh, &xmu = lds.xmu;
  auto &sux = lds.sux, &suy = lds.suy;
  const int nx = p.nx, ny = p.ny;
  const int c = threadIdx.x;
  const int gx = wrapc(X0 - 3 * M + c, nx);
  const bool col_out = c >= 3 * M && c < 3 * M + ncol && X0 + c - 3 * M < nx;
  const int cm = c > 0 ? c - 1 : 0, cp = c < BW - 1 ? c + 1 : BW - 1;  // edge lanes: values unused
  const size_t ns = (size_t)p.ns;
  const T *ux_g = u, *uy_g = u + ns;
  const T dt = T(p.dt), dtg = T(p.dt) * T(p.gamma);
  const T a = T(p.a), b = T(p.b), kappa = T(p.kappa), cQ = T(p.cQ), cC = T(p.cC);
  const int t0 = y0 - 3 * M, t1 = y1 + 4 * M - 1;  // iterations [t0, t1)
  const bool wide = ny >= 4 * M + 1;                // rows in [t0, t1] wrap at most once

  // substep s at iteration t: newest input row t-4s; registers hold
  // phi rows (t-4s-2, t-4s-1), h rows (t-4s-3, t-4s-2), mu rows (t-4s-4, t-4s-3),
  // and carry[s] = the row phi^s(t-4s) produced by substep s-1 last iteration
  T ph2[M], ph1[M], h2[M], h1[M], m2[M], m1[M], carry[M];
#pragma unroll
  for (int s = 0; s < M; s++) ph2[s] = ph1[s] = h2[s] = h1[s] = m2[s] = m1[s] = carry[s] = T(0);

  auto row_of = [&](int t) { return wide ? wrap1(t, ny) : wrapc(t, ny); };
  // input rows in flight: queue slot k holds row t0 + k + 2j at its j-th use
  T qphi[2], qux[2], quy[2];
#pragma unroll
  for (int k = 0; k < 2; k++) {
    qphi[k] = qux[k] = quy[k] = T(0);
    if (t0 + k < t1) {
      const int g = gx + nx * row_of(t0 + k);
      qphi[k] = phi_in[g];
      qux[k] = ux_g[g];
      quy[k] = uy_g[g];
    }
  }
  int slot = 0;                 // (t - t0) mod R, the ring row of input row t
  int rq = row_of(t0 + 2);      // lattice row of t + 2, the next refill
  // one iteration: input row t from queue slot k (parity of the published rows = k)
  auto iterate = [&](const int t, const int k) {
    const int par = k;
    // publish last iteration's rows and the new u* row
    sux[slot][c] = qux[k];
    suy[slot][c] = quy[k];
#pragma unroll
    for (int s = 0; s < M; s++) {
      xphi[par][s][c] = ph1[s];
      xh[par][s][c] = h1[s];
      xmu[par][s][c] = m1[s];
    }
    carry[0] = qphi[k];  // phi^0 row t
    if (t + 2 < t1) {    // refill the slot with row t + 2
      const int g = gx + nx * rq;
      qphi[k] = phi_in[g];
      qux[k] = ux_g[g];
      quy[k] = uy_g[g];
    }
    rq = rq + 1 == ny ? 0 : rq + 1;
    __syncthreads();
    T last = T(0);
    // substeps in reverse order: substep s reads carry[s] before substep s-1 replaces it
#pragma unroll
    for (int s = M - 1; s >= 0; s--) {
      // u* rows t-4s-2 (below), t-4s-1 (centre), t-4s (above) of the ring
      // (4s + 1 < R, so one correction brings the ring row into [0, R))
      int kc = slot - 4 * s - 1;
      kc += kc < 0 ? R : 0;
      const int kd = kc == 0 ? R - 1 : kc - 1, ku = kc == R - 1 ? 0 : kc + 1;
      // advection half-step at row t-4s-1
      const T pc = ph1[s], pdn = ph2[s], pup = carry[s];
      const T pw = xphi[par][s][cm], pe = xphi[par][s][cp];
      const T uxc = sux[kc][c], uxw = sux[kc][cm], uxe = sux[kc][cp];
      const T uyc = suy[kc][c], uyd = suy[kd][c], uyu = suy[ku][c];
      T rhs;
      if constexpr (!FLUX) {
        const T tx = pc * ((uxe - uxw) * T(0.5)) + upwind_diff(uxc, pw, pc, pe);
        const T ty = pc * ((uyu - uyd) * T(0.5)) + upwind_diff(uyc, pdn, pc, pup);
        rhs = tx + ty;
      } else {
        const T vxe = (uxc + uxe) * T(0.5), vxw = (uxw + uxc) * T(0.5);
        const T vyu = (uyc + uyu) * T(0.5), vyd = (uyd + uyc) * T(0.5);
        const T tx = upwind_flux(vxe, pc, pe) - upwind_flux(vxw, pw, pc);
        const T ty = upwind_flux(vyu, pc, pup) - upwind_flux(vyd, pdn, pc);
        rhs = tx + ty;
      }
      const T hn = pc - dt * rhs;
      // diffusion potential at row t-4s-2: a h + b phi^3 - kappa L h
      const T hc = h1[s];
      const T Lh = cQ * ((xh[par][s][cp] + xh[par][s][cm]) + (hn + h2[s])) + cC * hc;
      const T ps = ph2[s];
      const T mn = a * hc + b * ps * ps * ps - kappa * Lh;
      // phi^{s+1} at row t-4s-3: h + dt Gamma L mu
      const T mc = m1[s];
      const T Lm = cQ * ((xmu[par][s][cp] + xmu[par][s][cm]) + (mn + m2[s])) + cC * mc;
      const T out = h2[s] + dtg * Lm;
      // rotate this substep's rows
      ph2[s] = ph1[s];
      ph1[s] = carry[s];
      h2[s] = h1[s];
      h1[s] = hn;
      m2[s] = m1[s];
      m1[s] = mn;
      if (s + 1 < M) carry[s + 1] = out;
      else last = out;
    }
    const int yo = t - 4 * M + 1;  // row of the last substep's output
    if (col_out && yo >= y0 && yo < y1) phi_out[gx + nx * yo] = last;
    slot = slot + 1 == R ? 0 : slot + 1;
  };
  // unrolled by two so the queue slot and the parity are static
  for (int t = t0; t < t1; t += 2) {
    iterate(t, 0);
    if (t + 1 < t1) iterate(t + 1, 1);
  }
}

template <typename T, int M, int BW, bool FLUX>
__global__ void __launch_bounds__(BW) k_ch_march(KParams p, int seg, const T *__restrict__ phi_in,
                                                 const T *__restrict__ u, T *__restrict__ phi_out) {
  __shared__ MarchLds<T, M, BW> lds;
  int bx, by, bz;
  tile_coords(bx, by, bz);
  const int y0 = by * seg;
  ch_march_body<T, M, BW, FLUX>(lds, p, bx * (BW - 6 * M), BW - 6 * M, y0, min(y0 + seg, p.ny), phi_in, u,
                                phi_out);
}

// M substeps (one march) of the simulations of a group of a batch's substep
// launch: a tile is (simulation, X0, y0) with output columns [X0, X0 + ncol)
// and rows [y0, y0 + seg).  The tile table of a plan is blocked for the
// plan's largest fuse, so a group that fuses fewer substeps (the last ones
// of a simulation) uses the same table with M < fuse.
template <typename T, int M, int BW>
__global__ void __launch_bounds__(BW) k_chm_batch(const SimDesc *__restrict__ sims, const TileRef *__restrict__ tiles,
                                                  T *__restrict__ phi, const T *__restrict__ u, int par, int j,
                                                  int jpar, int seg, int ncol) {
  __shared__ MarchLds<T, M, BW> lds;  // one allocation for both advection forms
  int b, unused1, unused2;
  tile_coords(b, unused1, unused2);
  const TileRef tr = tiles[b];
  const SimDesc &sd = sims[tr.sim];
  const int src = batch_phi_buf(sd, par) ^ jpar;
  const int y1 = min(tr.y0 + seg, sd.p.ny);
  const T *in = phi + sd.phi[src];
  T *out = phi + sd.phi[1 - src];
  if (sd.p.advection == 1)
    ch_march_body<T, M, BW, true>(lds, sd.p, tr.x0, ncol, tr.y0, y1, in, u + sd.u, out);
  else
    ch_march_body<T, M, BW, false>(lds, sd.p, tr.x0, ncol, tr.y0, y1, in, u + sd.u, out);
}

// Geometry of the fused-tile kernel.  The staged box holds the tile plus a
// halo of H = 3M rows; in x the halo is rounded up to whole 16-byte vectors
// (HA), so that the box starts on a vector boundary of the lattice row and
// is staged and stored with 16-byte accesses.  LDS is the bytes of
// k_ch_tile's four arrays: two for phi, h and the diffusion potential, which
// rotate (see k_ch_tile), and u*_x, u*_y.
template <typename T, int M, int TO>
struct FusedTileGeom {
  static constexpr int V = 16 / (int)sizeof(T);  // elements per 16-byte vector
  static constexpr int H = 3 * M;
  static constexpr int HA = (H + V - 1) / V * V;
  static constexpr int L0 = TO + 2 * H;  // staged rows
  static constexpr int LW = TO + 2 * HA;  // staged columns, a multiple of V
  // Rows lie back to back in LDS (pitch LW): a wavefront's consecutive items
  // are then consecutive 16-byte vectors of LDS, which the 64 banks serve
  // without conflicts.
  static constexpr size_t LDS = 4ull * L0 * LW * sizeof(T);
};

// Rows [gy0, gy0 + NR) x columns [gx0, gx0 + NC * V) of a periodic 2D field
// staged in 16-byte vectors: issue() puts a thread's loads in flight,
// commit() writes them into an LDS array of row pitch P (column c at
// OFF + c).  gx0 is a multiple of V.  With `whole` (nx a multiple of V and
// an aligned field) every vector lies inside one lattice row, so one wrap
// per vector suffices; otherwise each element wraps on its own.
template <typename T, int NR, int NC, int NTH>
struct RowStage {
  static constexpr int V = 16 / (int)sizeof(T);
  static constexpr int N = NR * NC;
  static constexpr int K = (N + NTH - 1) / NTH;
  typedef T vec __attribute__((ext_vector_type(V)));
  vec v[K];

  __device__ __forceinline__ void issue(const T *__restrict__ f, int nx, int ny, int gx0, int gy0, bool whole) {
    const bool one = nx >= NC * V && ny >= NR;  // the box wraps at most once per axis
    auto wrap = [one](int a, int n) { return one ? wrap1(a, n) : wrapc(a, n); };
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      if (N % NTH == 0 || i < N) {
        const int r = i / NC, c = i % NC;
        const T *row = f + (size_t)nx * wrap(gy0 + r, ny);
        if (whole) {
          v[k] = *reinterpret_cast<const vec *>(row + wrap(gx0 + V * c, nx));
        } else {
#pragma unroll
          for (int j = 0; j < V; j++) v[k][j] = row[wrap(gx0 + V * c + j, nx)];
        }
      }
    }
  }
  template <int P, int OFF>
  __device__ __forceinline__ void commit(T *s) const {
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      if (N % NTH == 0 || i < N) *reinterpret_cast<vec *>(s + (i / NC) * P + OFF + V * (i % NC)) = v[k];
    }
  }
};

// Calls f(std::integral_constant<int, 0>{}) ... f(std::integral_constant<int, N - 1>{}) in order,
// so that f can use its argument as a constant expression.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// v of lane l - 1 (DIR = -1) or lane l + 1 (DIR = +1) of the wavefront, by a
// DPP whole-wave shift; lanes 0 and 63 receive 0 for DIR = -1 and +1.
template <int DIR, typename T>
__device__ __forceinline__ T lane_shift(T v) {
  constexpr int ctrl = DIR < 0 ? 0x138 : 0x130;  // wave_shr:1, wave_shl:1
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, 0xf, 0xf, false));
  } else {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), ctrl, 0xf, 0xf, false);
    return __builtin_bit_cast(T, (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)hi << 32));
  }
}

// M convection-diffusion substeps of one TO x TO tile in a single launch
// (2D; the standard 5-point Laplacian, or with LAP9 the 9-point one of weight
// cQ on the faces, cR on the diagonals and cC at the centre).  phi and u* are staged once with a halo
// of 3M; substep s then works on a region that shrinks by 3 on every side
// (its output region is the next substep's input), entirely in LDS: h with
// a halo of 2, the diffusion potential with a halo of 1, then phi^{s+1}.
// Global traffic: phi and u* read once, phi' written once.
// Two arrays A and B hold phi, h and the potential: with phi^s in A, h goes
// to B, the potential overwrites phi^s in A (its phase reads phi only at
// the site it writes) and phi^{s+1} overwrites h in B (likewise), after
// which A and B swap roles.
// A work item is V consecutive sites of a row (one 16-byte vector).  A phase
// runs over whole staged rows of its row range, so item i of a phase is the
// vector at offset r0 P + V i, and thread t takes items t, t + NTH, ...; the
// sites it computes in columns outside the region use values from outside
// the region and are never read by a site inside the next region.  Rows lie
// back to back in LDS, so a wavefront's 64 items are 1 KiB of consecutive
// LDS, read and written without bank conflicts.  (Regions of only their own
// columns took fewer instructions but made every row change inside a
// wavefront a bank conflict, and ran slower.)  The neighbour
// west (east) of a vector's first (last) site is the last (first) element
// of the vector in the previous (next) lane, which holds the previous (next)
// item, except at the edges of the wavefront: there it is read from LDS.
// The same holds for the rows above and below, whose edge values are the
// 9-point Laplacian's diagonal neighbours.  Every phase loop has
// a constant trip count and is unrolled, so that one item's loads can be
// issued under another's arithmetic.
// NTH threads per block (256, 512 or 1024).
template <typename T, int M, int TO, bool FLUX, int NTH, bool LAP9>
__global__ void __launch_bounds__(NTH) k_ch_tile(KParams p, const T *__restrict__ phi_in, const T *__restrict__ u,
                                                 T *__restrict__ phi_out) {
  using G = FusedTileGeom<T, M, TO>;
  constexpr int V = G::V, H = G::H, HA = G::HA, L0 = G::L0, LW = G::LW;
  constexpr int P = LW, NQ = LW / V;  // row pitch (rows back to back) and vectors per row
  static_assert(NTH % 64 == 0, "items of a wavefront are consecutive");
  typedef T vec __attribute__((ext_vector_type(V)));
  __shared__ __attribute__((aligned(16))) T sA[L0 * P], sB[L0 * P], sux[L0 * P], suy[L0 * P];
  int bx, by, bz;
  tile_coords(bx, by, bz);
  const int x0 = bx * TO, y0 = by * TO;
  const int nx = p.nx, ny = p.ny;
  const size_t ns = (size_t)p.ns;
  auto aligned = [](const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  // nx a multiple of V keeps every row start (and so every vector) aligned
  const bool whole = nx % V == 0 && aligned(phi_in) && aligned(u) && aligned(u + ns) && aligned(phi_out);
  {
    RowStage<T, L0, NQ, NTH> lphi, lux, luy;
    lphi.issue(phi_in, nx, ny, x0 - HA, y0 - H, whole);
    lux.issue(u, nx, ny, x0 - HA, y0 - H, whole);
    luy.issue(u + ns, nx, ny, x0 - HA, y0 - H, whole);
    lphi.template commit<P, 0>(sA);
    lux.template commit<P, 0>(sux);
    luy.template commit<P, 0>(suy);
  }
  __syncthreads();
  const T dt = T(p.dt), dtg = T(p.dt) * T(p.gamma);
  const T a = T(p.a), b = T(p.b), kappa = T(p.kappa), cQ = T(p.cQ), cR = T(p.cR), cC = T(p.cC);
  const int lane = threadIdx.x & 63;
  // a work item is the vector at element offset o of an array; the rows above
  // and below are at o - P and o + P
  auto ld = [](const T *arr, int o) { return *reinterpret_cast<const vec *>(arr + o); };
  auto st = [](T *arr, int o, vec v) { *reinterpret_cast<vec *>(arr + o) = v; };
  // the V-site neighbours to the west and east of the vector c at offset o of
  // arr: the neighbouring element is the last (first) of the previous (next)
  // item, held by the previous (next) lane, and read from LDS only at the
  // edges of the wavefront.  Every lane issues that LDS load (the others read
  // element 0, a broadcast), so no branch is formed around it.  At a row's
  // first (last) vector this is the last (first) element of the neighbouring
  // row: it feeds only the site in staged column 0 (LW - 1), which lies
  // outside every region.
  auto west = [&](const T *arr, vec c, int o) {
    const bool far = lane == 0;
    const T l = arr[far ? o - 1 : 0];
    const T d = lane_shift<-1>(c[V - 1]);
    vec r;
    r[0] = far ? l : d;
#pragma unroll
    for (int j = 1; j < V; j++) r[j] = c[j - 1];
    return r;
  };
  auto east = [&](const T *arr, vec c, int o) {
    const bool far = lane == 63;
    const T l = arr[far ? o + V : 0];
    const T d = lane_shift<+1>(c[0]);
    vec r;
#pragma unroll
    for (int j = 0; j < V - 1; j++) r[j] = c[j + 1];
    r[V - 1] = far ? l : d;
    return r;
  };
  // the items of rows [r0, r1): whole staged rows, item i at offset
  // r0 P + V i.  Rows r0 - 1 and r1 are inside the box (r0 >= 1, r1 <= L0 - 1).
  auto region = [](auto R0, auto R1, auto body) {
    constexpr int r0 = decltype(R0)::value, r1 = decltype(R1)::value;
    static_assert(r0 >= 1 && r1 <= L0 - 1, "neighbour rows inside the staged box");
    constexpr int N = (r1 - r0) * NQ, K = (N + NTH - 1) / NTH;
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      if (N % NTH == 0 || i < N) body(r0 * P + V * i);
    }
  };
  using std::integral_constant;

  static_for<M>([&](auto S) {
    constexpr int s = decltype(S)::value;
    T *const sp = s % 2 == 0 ? sA : sB;  // phi^s, then the potential
    T *const sq = s % 2 == 0 ? sB : sA;  // h, then phi^{s+1}
    constexpr int lo = 3 * s;
    // h on rows [lo + 1, L0 - lo - 1)
    region(integral_constant<int, lo + 1>{}, integral_constant<int, L0 - lo - 1>{}, [&](int o) {
      const vec pc = ld(sp, o), pdn = ld(sp, o - P), pup = ld(sp, o + P);
      const vec uxc = ld(sux, o);
      const vec uyc = ld(suy, o), uyd = ld(suy, o - P), uyu = ld(suy, o + P);
      const vec pw = west(sp, pc, o), pe = east(sp, pc, o);
      const vec uxw = west(sux, uxc, o), uxe = east(sux, uxc, o);
      vec h;
#pragma unroll
      for (int j = 0; j < V; j++) {
        T rhs;
        if constexpr (!FLUX) {
          const T tx =
              pc[j] * ((uxe[j] - uxw[j]) * T(0.5)) + uxc[j] * (uxc[j] > T(0) ? pc[j] - pw[j] : pe[j] - pc[j]);
          const T ty =
              pc[j] * ((uyu[j] - uyd[j]) * T(0.5)) + uyc[j] * (uyc[j] > T(0) ? pc[j] - pdn[j] : pup[j] - pc[j]);
          rhs = tx + ty;
        } else {
          const T vxe = (uxc[j] + uxe[j]) * T(0.5), vxw = (uxw[j] + uxc[j]) * T(0.5);
          const T vyu = (uyc[j] + uyu[j]) * T(0.5), vyd = (uyd[j] + uyc[j]) * T(0.5);
          const T tx = (vxe > T(0) ? vxe * pc[j] : vxe * pe[j]) - (vxw > T(0) ? vxw * pw[j] : vxw * pc[j]);
          const T ty = (vyu > T(0) ? vyu * pc[j] : vyu * pup[j]) - (vyd > T(0) ? vyd * pdn[j] : vyd * pc[j]);
          rhs = tx + ty;
        }
        h[j] = pc[j] - dt * rhs;
      }
      st(sq, o, h);
    });
    __syncthreads();
    // diffusion potential on [lo + 2, L0 - lo - 2), over phi^s
    region(integral_constant<int, lo + 2>{}, integral_constant<int, L0 - lo - 2>{}, [&](int o) {
      const vec hc = ld(sq, o), hdn = ld(sq, o - P), hup = ld(sq, o + P);
      const vec ph = ld(sp, o);
      const vec hw = west(sq, hc, o), he = east(sq, hc, o);
      vec dg;  // sums of the diagonal neighbours
      if constexpr (LAP9) {
        const vec dw = west(sq, hdn, o - P), de = east(sq, hdn, o - P);
        const vec uw = west(sq, hup, o + P), ue = east(sq, hup, o + P);
#pragma unroll
        for (int j = 0; j < V; j++) dg[j] = (ue[j] + uw[j]) + (de[j] + dw[j]);
      }
      vec mu;
#pragma unroll
      for (int j = 0; j < V; j++) {
        T Lh = cQ * ((he[j] + hw[j]) + (hup[j] + hdn[j])) + cC * hc[j];
        if constexpr (LAP9) Lh += cR * dg[j];
        mu[j] = a * hc[j] + b * ph[j] * ph[j] * ph[j] - kappa * Lh;
      }
      st(sp, o, mu);
    });
    __syncthreads();
    // phi^{s+1} on [lo + 3, L0 - lo - 3), over h
    region(integral_constant<int, lo + 3>{}, integral_constant<int, L0 - lo - 3>{}, [&](int o) {
      const vec mc = ld(sp, o), mdn = ld(sp, o - P), mup = ld(sp, o + P);
      const vec hc = ld(sq, o);
      const vec mw = west(sp, mc, o), me = east(sp, mc, o);
      vec dg;
      if constexpr (LAP9) {
        const vec dw = west(sp, mdn, o - P), de = east(sp, mdn, o - P);
        const vec uw = west(sp, mup, o + P), ue = east(sp, mup, o + P);
#pragma unroll
        for (int j = 0; j < V; j++) dg[j] = (ue[j] + uw[j]) + (de[j] + dw[j]);
      }
      vec out;
#pragma unroll
      for (int j = 0; j < V; j++) {
        T Lm = cQ * ((me[j] + mw[j]) + (mup[j] + mdn[j])) + cC * mc[j];
        if constexpr (LAP9) Lm += cR * dg[j];
        out[j] = hc[j] + dtg * Lm;
      }
      st(sq, o, out);
    });
    __syncthreads();
  });
  // phi^M is in B after an odd number of substeps, else in A
  const T *res = M % 2 == 1 ? sB : sA;
  constexpr int NO = TO / V;
  for (int i = threadIdx.x; i < TO * NO; i += NTH) {
    const int ty = i / NO, tx = V * (i % NO);
    const int x = x0 + tx, y = y0 + ty;
    if (y >= ny) continue;
    const vec v = ld(res, (H + ty) * P + HA + tx);
    if (whole) {
      if (x < nx) *reinterpret_cast<vec *>(phi_out + (size_t)nx * y + x) = v;
    } else {
#pragma unroll
      for (int j = 0; j < V; j++)
        if (x + j < nx) phi_out[(size_t)nx * y + x + j] = v[j];
    }
  }
}

// Items per thread of the fixed-mapping fused-tile kernel (k_ch_tile2): the
// staged box's vectors over NTH threads.
template <typename T, int M, int TO, int NTH>
struct FusedTile2 {
  using G = FusedTileGeom<T, M, TO>;
  static constexpr int NQ = G::LW / G::V;  // vectors per staged row
  static constexpr int NI = G::L0 * NQ;    // vectors of the staged box
  static constexpr int K = (NI + NTH - 1) / NTH;
  static constexpr size_t LDS = 2ull * G::L0 * G::LW * sizeof(T);
};

// M convection-diffusion substeps of a TO x TO tile in one launch, like
// k_ch_tile, with a fixed assignment of the staged box's vectors to threads:
// vector i (row i / NQ, column V (i % NQ)) belongs to thread i % NTH for the
// whole launch.  A phase reads the thread's own vector and the rows above
// and below from LDS; the east and west neighbours come from the
// neighbouring lanes (which own the neighbouring vectors of the row) by a
// DPP shift, and from LDS at the wavefront's edges.  u* is fixed over
// the substeps, so the advection half-step of each site is written once, in
// registers, as five coefficients,
//   h = c0 phi + cW phi_W + cE phi_E + cS phi_S + cN phi_N,
// which cover both the paper's form (Eqs. adv, centrdiff, backdiff, fordiff)
// and the flux form; u* is staged through LDS only to form them.  Two LDS
// arrays rotate as in k_ch_tile: with phi^s in A, h goes to B, the potential
// to A and phi^{s+1} to B.  A phase runs over whole rows of its region;
// the values it computes at columns outside the region are never read by
// a site inside it.  phi^M leaves from registers.  The coefficients take
// 5 V registers per vector, so at most three vectors per thread.
template <typename T, int M, int TO, int NTH, bool LAP9>
__global__ void __launch_bounds__(NTH) k_ch_tile2(KParams p, const T *__restrict__ phi_in, const T *__restrict__ u,
                                                  T *__restrict__ phi_out) {
  using G = FusedTileGeom<T, M, TO>;
  using F2 = FusedTile2<T, M, TO, NTH>;
  constexpr int V = G::V, H = G::H, HA = G::HA, L0 = G::L0, P = G::LW;  // rows back to back
  constexpr int NQ = F2::NQ, NI = F2::NI, K = F2::K;
  static_assert(NTH % 64 == 0, "vectors of a wavefront are consecutive");
  typedef T vec __attribute__((ext_vector_type(V)));
  __shared__ __attribute__((aligned(16))) T sA[L0 * P], sB[L0 * P];
  int bx, by, bz;
  tile_coords(bx, by, bz);
  const int x0 = bx * TO, y0 = by * TO;
  const int nx = p.nx, ny = p.ny;
  const size_t ns = (size_t)p.ns;
  auto aligned = [](const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  const bool whole = nx % V == 0 && aligned(phi_in) && aligned(u) && aligned(u + ns) && aligned(phi_out);
  const bool one = nx >= G::LW && ny >= L0;  // the box wraps at most once per axis
  const int lane = threadIdx.x & 63;
  auto ld = [](const T *arr, int y, int x) { return *reinterpret_cast<const vec *>(arr + y * P + x); };
  auto st = [](T *arr, int y, int x, vec v) { *reinterpret_cast<vec *>(arr + y * P + x) = v; };
  // the neighbouring element comes from the neighbouring lane, which holds
  // the previous (next) vector of the box, and from LDS at the wavefront's
  // edges.  At a row's first (last) vector it is the last (first) element of
  // the neighbouring row (clamped to the box at its first and last vector):
  // it feeds only the site in staged column 0 (LW - 1), outside every region.
  auto west = [&](const T *arr, vec c, int y, int x) {
    const bool far = lane == 0;
    const T l = arr[far ? max(y * P + x - 1, 0) : 0];
    const T d = lane_shift<-1>(c[V - 1]);
    vec r;
    r[0] = far ? l : d;
#pragma unroll
    for (int j = 1; j < V; j++) r[j] = c[j - 1];
    return r;
  };
  auto east = [&](const T *arr, vec c, int y, int x) {
    const bool far = lane == 63;
    const T l = arr[far ? min(y * P + x + V, L0 * P - 1) : 0];
    const T d = lane_shift<+1>(c[0]);
    vec r;
#pragma unroll
    for (int j = 0; j < V - 1; j++) r[j] = c[j + 1];
    r[V - 1] = far ? l : d;
    return r;
  };
  auto load_vec = [&](const T *f, int r, int q) {
    const int gy = one ? wrap1(y0 - H + r, ny) : wrapc(y0 - H + r, ny);
    const T *row = f + (size_t)nx * gy;
    const int gx = x0 - HA + V * q;
    vec v;
    if (whole) {
      v = *reinterpret_cast<const vec *>(row + (one ? wrap1(gx, nx) : wrapc(gx, nx)));
    } else {
#pragma unroll
      for (int j = 0; j < V; j++) v[j] = row[one ? wrap1(gx + j, nx) : wrapc(gx + j, nx)];
    }
    return v;
  };

  vec ph[K], c0[K], cw[K], ce[K], cs[K], cn[K];
  {
    // u* through LDS; phi stays in flight in registers meanwhile
    vec ux[K], uy[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      if (NI % NTH == 0 || i < NI) {
        ux[k] = load_vec(u, i / NQ, i % NQ);
        uy[k] = load_vec(u + ns, i / NQ, i % NQ);
        ph[k] = load_vec(phi_in, i / NQ, i % NQ);
      }
    }
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      if (NI % NTH == 0 || i < NI) {
        st(sA, i / NQ, V * (i % NQ), ux[k]);
        st(sB, i / NQ, V * (i % NQ), uy[k]);
      }
    }
    __syncthreads();
    const T dt = T(p.dt);
    const bool flux = p.advection == 1;
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      const int r = (NI % NTH == 0 || i < NI) ? i / NQ : 0, x = V * (i % NQ);
      // every lane of a wavefront takes part in the shifts; rows without
      // both neighbours in the box only produce unused coefficients
      const vec uxc = ld(sA, r, x);
      const vec uw = west(sA, uxc, r, x), ue = east(sA, uxc, r, x);
      if ((NI % NTH == 0 || i < NI) && r >= 1 && r < L0 - 1) {
        const vec uyc = ld(sB, r, x), un = ld(sB, r + 1, x), us = ld(sB, r - 1, x);
#pragma unroll
        for (int j = 0; j < V; j++) {
          const T vx = uxc[j], vy = uyc[j];
          if (!flux) {
            const T div = (ue[j] - uw[j]) * T(0.5) + (un[j] - us[j]) * T(0.5);
            const T a_w = vx > T(0) ? dt * vx : T(0), a_e = vx > T(0) ? T(0) : -dt * vx;
            const T a_s = vy > T(0) ? dt * vy : T(0), a_n = vy > T(0) ? T(0) : -dt * vy;
            cw[k][j] = a_w;
            ce[k][j] = a_e;
            cs[k][j] = a_s;
            cn[k][j] = a_n;
            c0[k][j] = T(1) - dt * div - ((a_w + a_e) + (a_s + a_n));
          } else {
            const T ve = (vx + ue[j]) * T(0.5), vw = (uw[j] + vx) * T(0.5);
            const T vn = (vy + un[j]) * T(0.5), vs = (us[j] + vy) * T(0.5);
            const T pe = ve > T(0) ? ve : T(0), me = ve > T(0) ? T(0) : ve;
            const T pw = vw > T(0) ? vw : T(0), mw = vw > T(0) ? T(0) : vw;
            const T pn = vn > T(0) ? vn : T(0), mn = vn > T(0) ? T(0) : vn;
            const T ps = vs > T(0) ? vs : T(0), msv = vs > T(0) ? T(0) : vs;
            cw[k][j] = dt * pw;
            ce[k][j] = -dt * me;
            cs[k][j] = dt * ps;
            cn[k][j] = -dt * mn;
            c0[k][j] = T(1) - dt * ((pe - mw) + (pn - msv));
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int i = threadIdx.x + k * NTH;
    if (NI % NTH == 0 || i < NI) st(sA, i / NQ, V * (i % NQ), ph[k]);
  }
  __syncthreads();
  const T dtg = T(p.dt) * T(p.gamma);
  const T a = T(p.a), b = T(p.b), kappa = T(p.kappa), cQ = T(p.cQ), cR = T(p.cR), cC = T(p.cC);
  // the sums of the four diagonal neighbours of a vector with rows n (above)
  // and s (below) of array arr
  auto diag = [&](const T *arr, vec n, vec s, int r, int x) {
    const vec nw = west(arr, n, r + 1, x), ne = east(arr, n, r + 1, x);
    const vec sw = west(arr, s, r - 1, x), se = east(arr, s, r - 1, x);
    vec dg;
#pragma unroll
    for (int j = 0; j < V; j++) dg[j] = (ne[j] + nw[j]) + (se[j] + sw[j]);
    return dg;
  };
  static_for<M>([&](auto S) {
    constexpr int s = decltype(S)::value;
    T *const sp = s % 2 == 0 ? sA : sB;  // phi^s, then the potential
    T *const sq = s % 2 == 0 ? sB : sA;  // h, then phi^{s+1}
    constexpr int lo = 3 * s;
    // h on rows [lo + 1, L0 - lo - 1)
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      // vectors past the box (the last slot) compute at row 0 and are discarded
      const int r = (NI % NTH == 0 || i < NI) ? i / NQ : 0, x = V * (i % NQ);
      if (k * NTH + NTH - 1 < (lo + 1) * NQ || k * NTH >= (L0 - lo - 1) * NQ) continue;  // no row of this slot
      const bool in = (NI % NTH == 0 || i < NI) && r >= lo + 1 && r < L0 - lo - 1;
      const vec pc = ld(sp, r, x);
      const vec pw = west(sp, pc, r, x), pe = east(sp, pc, r, x);
      if (in) {
        const vec pn = ld(sp, r + 1, x), ps = ld(sp, r - 1, x);
        vec hv;
#pragma unroll
        for (int j = 0; j < V; j++)
          hv[j] = c0[k][j] * pc[j] + cw[k][j] * pw[j] + ce[k][j] * pe[j] + cs[k][j] * ps[j] + cn[k][j] * pn[j];
        st(sq, r, x, hv);
      }
      if constexpr (K > 2) __builtin_amdgcn_sched_barrier(0);  // one vector's temporaries at a time
    }
    __syncthreads();
    // diffusion potential on [lo + 2, L0 - lo - 2), over phi^s
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      // vectors past the box (the last slot) compute at row 0 and are discarded
      const int r = (NI % NTH == 0 || i < NI) ? i / NQ : 0, x = V * (i % NQ);
      if (k * NTH + NTH - 1 < (lo + 2) * NQ || k * NTH >= (L0 - lo - 2) * NQ) continue;
      const bool in = (NI % NTH == 0 || i < NI) && r >= lo + 2 && r < L0 - lo - 2;
      const vec hc = ld(sq, r, x);
      const vec hw = west(sq, hc, r, x), he = east(sq, hc, r, x);
      const vec hn = ld(sq, in ? r + 1 : 0, x), hs = ld(sq, in ? r - 1 : 0, x);
      vec dg;
      if constexpr (LAP9) dg = diag(sq, hn, hs, in ? r : 1, x);
      if (in) {
        const vec pc = ld(sp, r, x);  // phi^s at this vector, overwritten below
        vec pt;
#pragma unroll
        for (int j = 0; j < V; j++) {
          T Lh = cQ * ((he[j] + hw[j]) + (hn[j] + hs[j])) + cC * hc[j];
          if constexpr (LAP9) Lh += cR * dg[j];
          pt[j] = a * hc[j] + b * pc[j] * pc[j] * pc[j] - kappa * Lh;
        }
        st(sp, r, x, pt);
      }
      if constexpr (K > 2) __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    // phi^{s+1} on [lo + 3, L0 - lo - 3), over h
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + k * NTH;
      // vectors past the box (the last slot) compute at row 0 and are discarded
      const int r = (NI % NTH == 0 || i < NI) ? i / NQ : 0, x = V * (i % NQ);
      if (k * NTH + NTH - 1 < (lo + 3) * NQ || k * NTH >= (L0 - lo - 3) * NQ) continue;
      const bool in = (NI % NTH == 0 || i < NI) && r >= lo + 3 && r < L0 - lo - 3;
      const vec mc = ld(sp, r, x);
      const vec mw = west(sp, mc, r, x), me = east(sp, mc, r, x);
      const vec mn = ld(sp, in ? r + 1 : 0, x), ms = ld(sp, in ? r - 1 : 0, x);
      vec dg;
      if constexpr (LAP9) dg = diag(sp, mn, ms, in ? r : 1, x);
      if (in) {
        const vec hc = ld(sq, r, x);  // h at this vector, overwritten below
        vec out;
#pragma unroll
        for (int j = 0; j < V; j++) {
          T Lm = cQ * ((me[j] + mw[j]) + (mn[j] + ms[j])) + cC * mc[j];
          if constexpr (LAP9) Lm += cR * dg[j];
          out[j] = hc[j] + dtg * Lm;
        }
        if constexpr (s + 1 < M) st(sq, r, x, out);
        else ph[k] = out;
      }
      if constexpr (K > 2) __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (s + 1 < M) __syncthreads();
  });
  // phi^M of the tile leaves from registers
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int i = threadIdx.x + k * NTH;
    const int r = i / NQ, q = i % NQ;
    if (!(NI % NTH == 0 || i < NI) || r < H || r >= H + TO || V * q < HA || V * q >= HA + TO) continue;
    const int y = y0 + r - H, x = x0 + V * q - HA;
    if (y >= ny) continue;
    if (whole) {
      if (x < nx) *reinterpret_cast<vec *>(phi_out + (size_t)nx * y + x) = ph[k];
    } else {
#pragma unroll
      for (int j = 0; j < V; j++)
        if (x + j < nx) phi_out[(size_t)nx * y + x + j] = ph[k][j];
    }
  }
}

// One convection-diffusion substep in 3D (standard 7-point Laplacian),
// marching along z.  A block of TXI x TYT threads owns TXI x 2 TYT (x, y)
// columns, two neighbouring rows per thread, and walks the z planes of its
// segment; the output is the middle (TXI - 6) x (2 TYT - 6) columns.  Per
// column the last planes of phi, h, the diffusion potential and u*_z live in
// registers (the z neighbours); x and y neighbours come from one LDS plane
// per quantity (phi, h, potential, u*_x, u*_y) published at the start of an
// iteration, except the y neighbour shared by a thread's two rows, which
// stays in registers.  The output plane trails the input plane by 3.  One
// barrier per plane; phi and u* are read once and phi' written once.
template <typename T, int TXI, int TYT, bool FLUX>
__global__ void __launch_bounds__(TXI *TYT) k_ch_march3(KParams p, int seg, const T *__restrict__ phi_in,
                                                        const T *__restrict__ u, T *__restrict__ phi_out) {
  constexpr int TYI = 2 * TYT;
  __shared__ T xphi[2][TYI][TXI], xh[2][TYI][TXI], xmu[2][TYI][TXI], xux[2][TYI][TXI], xuy[2][TYI][TXI];
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int cx = threadIdx.x % TXI, ty = threadIdx.x / TXI;
  const int cy0 = 2 * ty, cy1 = 2 * ty + 1;
  int bx, by, bz;
  tile_coords(bx, by, bz);
  const int X0 = bx * (TXI - 6), Y0 = by * (TYI - 6);
  const int z0 = bz * seg, z1 = min(z0 + seg, nz);
  const int gx = wrapc(X0 - 3 + cx, nx);
  const int gy0 = wrapc(Y0 - 3 + cy0, ny), gy1 = wrapc(Y0 - 3 + cy1, ny);
  const bool xin = cx >= 3 && cx < TXI - 3 && X0 + cx - 3 < nx;
  const bool out0 = xin && cy0 >= 3 && cy0 < TYI - 3 && Y0 + cy0 - 3 < ny;
  const bool out1 = xin && cy1 >= 3 && cy1 < TYI - 3 && Y0 + cy1 - 3 < ny;
  // edge lanes read themselves; their results are never used
  const int cxm = cx > 0 ? cx - 1 : 0, cxp = cx < TXI - 1 ? cx + 1 : TXI - 1;
  const int cym = cy0 > 0 ? cy0 - 1 : 0, cyp = cy1 < TYI - 1 ? cy1 + 1 : TYI - 1;
  const size_t ns = (size_t)p.ns;
  const T *ux_g = u, *uy_g = u + ns, *uz_g = u + 2 * ns;
  const T dt = T(p.dt), dtg = T(p.dt) * T(p.gamma);
  const T a = T(p.a), b = T(p.b), kappa = T(p.kappa), cQ = T(p.cQ), cC = T(p.cC);
  const int t0 = z0 - 3, t1 = z1 + 3;  // iterations [t0, t1); output plane t - 3
  const bool wide = nz >= 4;
  const size_t plane = (size_t)nx * ny;
  const size_t col0 = gx + (size_t)nx * gy0, col1 = gx + (size_t)nx * gy1;
  auto plane_of = [&](int t) { return wide ? wrap1(t, nz) : wrapc(t, nz); };
  int zq = plane_of(t0 + 2);  // lattice plane of t + 2, the next refill

  // per row r of the pair: phi planes (t-2, t-1), h (t-3, t-2), mu (t-4, t-3),
  // u*_x, u*_y at plane t-1, u*_z planes (t-2, t-1), and the loaded plane t
  T ph2[2] = {0, 0}, ph1[2] = {0, 0}, h2[2] = {0, 0}, h1[2] = {0, 0}, m2[2] = {0, 0}, m1[2] = {0, 0};
  T ux1[2] = {0, 0}, uy1[2] = {0, 0}, uz2[2] = {0, 0}, uz1[2] = {0, 0};
  // input planes in flight: queue slot k holds plane t0 + k + 2j at its j-th use
  T qphi[2][2], qux[2][2], quy[2][2], quz[2][2];
#pragma unroll
  for (int k = 0; k < 2; k++) {
    if (t0 + k < t1) {
      const size_t pz = plane * plane_of(t0 + k);
      qphi[k][0] = phi_in[col0 + pz];
      qux[k][0] = ux_g[col0 + pz];
      quy[k][0] = uy_g[col0 + pz];
      quz[k][0] = uz_g[col0 + pz];
      qphi[k][1] = phi_in[col1 + pz];
      qux[k][1] = ux_g[col1 + pz];
      quy[k][1] = uy_g[col1 + pz];
      quz[k][1] = uz_g[col1 + pz];
    }
  }
  // one iteration: input plane t from queue slot k (parity of the published planes = k)
  auto iterate = [&](const int t, const int k) {
    const int par = k;
    const int cy[2] = {cy0, cy1};
#pragma unroll
    for (int r = 0; r < 2; r++) {
      xphi[par][cy[r]][cx] = ph1[r];
      xh[par][cy[r]][cx] = h1[r];
      xmu[par][cy[r]][cx] = m1[r];
      xux[par][cy[r]][cx] = ux1[r];
      xuy[par][cy[r]][cx] = uy1[r];
    }
    T in[2], inux[2], inuy[2], inuz[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
      in[r] = qphi[k][r];
      inux[r] = qux[k][r];
      inuy[r] = quy[k][r];
      inuz[r] = quz[k][r];
    }
    if (t + 2 < t1) {  // refill the slot with plane t + 2
      const size_t pz = plane * zq;
      qphi[k][0] = phi_in[col0 + pz];
      qux[k][0] = ux_g[col0 + pz];
      quy[k][0] = uy_g[col0 + pz];
      quz[k][0] = uz_g[col0 + pz];
      qphi[k][1] = phi_in[col1 + pz];
      qux[k][1] = ux_g[col1 + pz];
      quy[k][1] = uy_g[col1 + pz];
      quz[k][1] = uz_g[col1 + pz];
    }
    zq = zq + 1 == nz ? 0 : zq + 1;
    __syncthreads();
    // y neighbours at the published plane: below row 0 and above row 1 from LDS,
    // between the two rows from registers
    const T phs = xphi[par][cym][cx], phn = xphi[par][cyp][cx];
    const T hs = xh[par][cym][cx], hnb = xh[par][cyp][cx];
    const T ms = xmu[par][cym][cx], mnb = xmu[par][cyp][cx];
    const T uys = xuy[par][cym][cx], uyn = xuy[par][cyp][cx];
    T out[2], hnew[2], mnew[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
      const int y = cy[r];
      // values of the neighbouring rows (south, north) in this plane
      const T p_s = r == 0 ? phs : ph1[0], p_n = r == 0 ? ph1[1] : phn;
      const T h_s = r == 0 ? hs : h1[0], h_n = r == 0 ? h1[1] : hnb;
      const T m_s = r == 0 ? ms : m1[0], m_n = r == 0 ? m1[1] : mnb;
      const T uy_s = r == 0 ? uys : uy1[0], uy_n = r == 0 ? uy1[1] : uyn;
      // advection half-step at plane t-1
      const T pc = ph1[r];
      const T pw = xphi[par][y][cxm], pe = xphi[par][y][cxp];
      const T pd = ph2[r], pu = in[r];
      const T uxc = ux1[r], uxw = xux[par][y][cxm], uxe = xux[par][y][cxp];
      const T uyc = uy1[r];
      const T uzc = uz1[r], uzd = uz2[r], uzu = inuz[r];
      T rhs;
      if constexpr (!FLUX) {
        const T tx = pc * ((uxe - uxw) * T(0.5)) + upwind_diff(uxc, pw, pc, pe);
        const T ty_ = pc * ((uy_n - uy_s) * T(0.5)) + upwind_diff(uyc, p_s, pc, p_n);
        const T tz = pc * ((uzu - uzd) * T(0.5)) + upwind_diff(uzc, pd, pc, pu);
        rhs = tx + ty_ + tz;
      } else {
        const T vxe = (uxc + uxe) * T(0.5), vxw = (uxw + uxc) * T(0.5);
        const T vyn = (uyc + uy_n) * T(0.5), vys = (uy_s + uyc) * T(0.5);
        const T vzu = (uzc + uzu) * T(0.5), vzd = (uzd + uzc) * T(0.5);
        const T tx = upwind_flux(vxe, pc, pe) - upwind_flux(vxw, pw, pc);
        const T ty_ = upwind_flux(vyn, pc, p_n) - upwind_flux(vys, p_s, pc);
        const T tz = upwind_flux(vzu, pc, pu) - upwind_flux(vzd, pd, pc);
        rhs = tx + ty_ + tz;
      }
      hnew[r] = pc - dt * rhs;
      // diffusion potential at plane t-2
      const T hc = h1[r];
      const T Lh = cQ * ((xh[par][y][cxp] + xh[par][y][cxm]) + (h_n + h_s) + (hnew[r] + h2[r])) + cC * hc;
      mnew[r] = a * hc + b * ph2[r] * ph2[r] * ph2[r] - kappa * Lh;
      // phi' at plane t-3
      const T mc = m1[r];
      const T Lm = cQ * ((xmu[par][y][cxp] + xmu[par][y][cxm]) + (m_n + m_s) + (mnew[r] + m2[r])) + cC * mc;
      out[r] = h2[r] + dtg * Lm;
    }
#pragma unroll
    for (int r = 0; r < 2; r++) {
      ph2[r] = ph1[r];
      ph1[r] = in[r];
      h2[r] = h1[r];
      h1[r] = hnew[r];
      m2[r] = m1[r];
      m1[r] = mnew[r];
      ux1[r] = inux[r];
      uy1[r] = inuy[r];
      uz2[r] = uz1[r];
      uz1[r] = inuz[r];
    }
    const int zo = t - 3;
    if (zo >= z0 && zo < z1) {
      if (out0) phi_out[col0 + plane * zo] = out[0];
      if (out1) phi_out[col1 + plane * zo] = out[1];
    }
  };
  // unrolled by two so the queue slot and the parity are static
  for (int t = t0; t < t1; t += 2) {
    iterate(t, 0);
    if (t + 1 < t1) iterate(t + 1, 1);
  }
}

// One convection-diffusion substep in 3D with the general 19-point Laplacian
// of the C14 form (weight cQ on the 6 faces, cR on the 12 edges, cC at the
// centre; cd_Q != 1), marching along z with the thread layout of
// k_ch_march3.  The Laplacian of a plane needs the in-plane neighbours of
// the planes above and below it, so the pipeline lags further: iteration t
// (input plane t) forms h at plane t-1 by the advection half-step, the
// diffusion potential at plane t-3 from h on planes t-4 .. t-2, and phi' at
// plane t-5 from the potential on planes t-6 .. t-4.  Every plane those two
// Laplacians read was formed in an earlier iteration: h and the potential
// are published into rings of four LDS planes (an iteration reads the two
// newest, the next one overwrites the oldest), so one barrier per plane
// still suffices.  With F(p) the sum over the 4 in-plane face neighbours
// and E(p) over the 4 in-plane diagonal neighbours of a column on plane p,
//   L q(p) = cQ [F(p) + q(p-1) + q(p+1)] + cR [E(p) + F(p-1) + F(p+1)] + cC q(p),
// so F of each plane is formed once, when the plane is newest, and kept in
// registers for the two later Laplacians that use it.
template <typename T, int TXI, int TYT, bool FLUX>
__global__ void __launch_bounds__(TXI *TYT) k_ch_march3w(KParams p, int seg, const T *__restrict__ phi_in,
                                                         const T *__restrict__ u, T *__restrict__ phi_out) {
  constexpr int TYI = 2 * TYT;
  __shared__ T xphi[2][TYI][TXI], xux[2][TYI][TXI], xuy[2][TYI][TXI], rh[4][TYI][TXI], rm[4][TYI][TXI];
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int cx = threadIdx.x % TXI, ty = threadIdx.x / TXI;
  const int cy0 = 2 * ty, cy1 = 2 * ty + 1;
  int bx, by, bz;
  tile_coords(bx, by, bz);
  const int X0 = bx * (TXI - 6), Y0 = by * (TYI - 6);
  const int z0 = bz * seg, z1 = min(z0 + seg, nz);
  const int gx = wrapc(X0 - 3 + cx, nx);
  const int gy0 = wrapc(Y0 - 3 + cy0, ny), gy1 = wrapc(Y0 - 3 + cy1, ny);
  const bool xin = cx >= 3 && cx < TXI - 3 && X0 + cx - 3 < nx;
  const bool out0 = xin && cy0 >= 3 && cy0 < TYI - 3 && Y0 + cy0 - 3 < ny;
  const bool out1 = xin && cy1 >= 3 && cy1 < TYI - 3 && Y0 + cy1 - 3 < ny;
  // edge lanes read themselves; their results are never used
  const int cxm = cx > 0 ? cx - 1 : 0, cxp = cx < TXI - 1 ? cx + 1 : TXI - 1;
  const int cym = cy0 > 0 ? cy0 - 1 : 0, cyp = cy1 < TYI - 1 ? cy1 + 1 : TYI - 1;
  const size_t ns = (size_t)p.ns;
  const T *ux_g = u, *uy_g = u + ns, *uz_g = u + 2 * ns;
  const T dt = T(p.dt), dtg = T(p.dt) * T(p.gamma);
  const T a = T(p.a), b = T(p.b), kappa = T(p.kappa), cQ = T(p.cQ), cR = T(p.cR), cC = T(p.cC);
  const int t0 = z0 - 3, t1 = z1 + 5;  // iterations [t0, t1); output plane t - 5
  const bool wide = nz >= 4;
  const size_t plane = (size_t)nx * ny;
  const size_t col0 = gx + (size_t)nx * gy0, col1 = gx + (size_t)nx * gy1;
  auto plane_of = [&](int t) { return wide ? wrap1(t, nz) : wrapc(t, nz); };
  int zq = plane_of(t0 + 2);  // lattice plane of t + 2, the next refill

  // per row r of the pair: phi planes t-1, t-2, t-3; u*_x, u*_y at t-1; u*_z
  // at t-2, t-1; h at t-2 .. t-5 and F_h at t-3, t-4; the potential at
  // t-4 .. t-6 and F_mu at t-5, t-6
  T ph1[2] = {0, 0}, ph2[2] = {0, 0}, ph3[2] = {0, 0};
  T ux1[2] = {0, 0}, uy1[2] = {0, 0}, uz2[2] = {0, 0}, uz1[2] = {0, 0};
  T h2[2] = {0, 0}, h3[2] = {0, 0}, h4[2] = {0, 0}, h5[2] = {0, 0}, fh3[2] = {0, 0}, fh4[2] = {0, 0};
  T m4[2] = {0, 0}, m5[2] = {0, 0}, m6[2] = {0, 0}, fm5[2] = {0, 0}, fm6[2] = {0, 0};
  // input planes in flight: queue slot k holds plane t0 + k + 2j at its j-th use
  T qphi[2][2], qux[2][2], quy[2][2], quz[2][2];
#pragma unroll
  for (int k = 0; k < 2; k++) {
    if (t0 + k < t1) {
      const size_t pz = plane * plane_of(t0 + k);
      qphi[k][0] = phi_in[col0 + pz];
      qux[k][0] = ux_g[col0 + pz];
      quy[k][0] = uy_g[col0 + pz];
      quz[k][0] = uz_g[col0 + pz];
      qphi[k][1] = phi_in[col1 + pz];
      qux[k][1] = ux_g[col1 + pz];
      quy[k][1] = uy_g[col1 + pz];
      quz[k][1] = uz_g[col1 + pz];
    }
  }
  // in-plane face sum and diagonal sum of a ring plane at both rows of the
  // pair; q0, q1 are this thread's own values of that plane
  auto face = [&](const T (&r)[TYI][TXI], const T q0, const T q1, T f[2]) {
    f[0] = (r[cy0][cxp] + r[cy0][cxm]) + (q1 + r[cym][cx]);
    f[1] = (r[cy1][cxp] + r[cy1][cxm]) + (r[cyp][cx] + q0);
  };
  auto diag = [&](const T (&r)[TYI][TXI], T e[2]) {
    const T s_m = r[cym][cxp] + r[cym][cxm], s_0 = r[cy0][cxp] + r[cy0][cxm];
    const T s_1 = r[cy1][cxp] + r[cy1][cxm], s_p = r[cyp][cxp] + r[cyp][cxm];
    e[0] = s_1 + s_m;
    e[1] = s_p + s_0;
  };
  // one iteration: input plane t from queue slot k (parity of the published planes = k)
  auto iterate = [&](const int t, const int k) {
    const int par = k;
    const int cy[2] = {cy0, cy1};
    const int sh = (t - 2) & 3, shp = (t - 3) & 3;  // ring planes of h at t-2, t-3
    const int sm = (t - 4) & 3, smp = (t - 5) & 3;  // ring planes of mu at t-4, t-5
#pragma unroll
    for (int r = 0; r < 2; r++) {
      xphi[par][cy[r]][cx] = ph1[r];
      xux[par][cy[r]][cx] = ux1[r];
      xuy[par][cy[r]][cx] = uy1[r];
      rh[sh][cy[r]][cx] = h2[r];
      rm[sm][cy[r]][cx] = m4[r];
    }
    T in[2], inux[2], inuy[2], inuz[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
      in[r] = qphi[k][r];
      inux[r] = qux[k][r];
      inuy[r] = quy[k][r];
      inuz[r] = quz[k][r];
    }
    if (t + 2 < t1) {  // refill the slot with plane t + 2
      const size_t pz = plane * zq;
      qphi[k][0] = phi_in[col0 + pz];
      qux[k][0] = ux_g[col0 + pz];
      quy[k][0] = uy_g[col0 + pz];
      quz[k][0] = uz_g[col0 + pz];
      qphi[k][1] = phi_in[col1 + pz];
      qux[k][1] = ux_g[col1 + pz];
      quy[k][1] = uy_g[col1 + pz];
      quz[k][1] = uz_g[col1 + pz];
    }
    zq = zq + 1 == nz ? 0 : zq + 1;
    __syncthreads();
    // advection half-step at plane t-1 (face neighbours only)
    const T phs = xphi[par][cym][cx], phn = xphi[par][cyp][cx];
    const T uys = xuy[par][cym][cx], uyn = xuy[par][cyp][cx];
    T hnew[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
      const int y = cy[r];
      const T p_s = r == 0 ? phs : ph1[0], p_n = r == 0 ? ph1[1] : phn;
      const T uy_s = r == 0 ? uys : uy1[0], uy_n = r == 0 ? uy1[1] : uyn;
      const T pc = ph1[r];
      const T pw = xphi[par][y][cxm], pe = xphi[par][y][cxp];
      const T pd = ph2[r], pu = in[r];
      const T uxc = ux1[r], uxw = xux[par][y][cxm], uxe = xux[par][y][cxp];
      const T uyc = uy1[r];
      const T uzc = uz1[r], uzd = uz2[r], uzu = inuz[r];
      T rhs;
      if constexpr (!FLUX) {
        const T tx = pc * ((uxe - uxw) * T(0.5)) + upwind_diff(uxc, pw, pc, pe);
        const T ty_ = pc * ((uy_n - uy_s) * T(0.5)) + upwind_diff(uyc, p_s, pc, p_n);
        const T tz = pc * ((uzu - uzd) * T(0.5)) + upwind_diff(uzc, pd, pc, pu);
        rhs = tx + ty_ + tz;
      } else {
        const T vxe = (uxc + uxe) * T(0.5), vxw = (uxw + uxc) * T(0.5);
        const T vyn = (uyc + uy_n) * T(0.5), vys = (uy_s + uyc) * T(0.5);
        const T vzu = (uzc + uzu) * T(0.5), vzd = (uzd + uzc) * T(0.5);
        const T tx = upwind_flux(vxe, pc, pe) - upwind_flux(vxw, pw, pc);
        const T ty_ = upwind_flux(vyn, pc, p_n) - upwind_flux(vys, p_s, pc);
        const T tz = upwind_flux(vzu, pc, pu) - upwind_flux(vzd, pd, pc);
        rhs = tx + ty_ + tz;
      }
      hnew[r] = pc - dt * rhs;
    }
    // the potential at plane t-3 from h on planes t-4 .. t-2
    T fh2[2], eh3[2], mnew[2];
    face(rh[sh], h2[0], h2[1], fh2);
    diag(rh[shp], eh3);
#pragma unroll
    for (int r = 0; r < 2; r++) {
      const T Lh = cQ * (fh3[r] + (h2[r] + h4[r])) + cR * (eh3[r] + (fh2[r] + fh4[r])) + cC * h3[r];
      mnew[r] = a * h3[r] + b * ph3[r] * ph3[r] * ph3[r] - kappa * Lh;
    }
    // phi' at plane t-5 from the potential on planes t-6 .. t-4
    T fm4[2], em5[2], out[2];
    face(rm[sm], m4[0], m4[1], fm4);
    diag(rm[smp], em5);
#pragma unroll
    for (int r = 0; r < 2; r++) {
      const T Lm = cQ * (fm5[r] + (m4[r] + m6[r])) + cR * (em5[r] + (fm4[r] + fm6[r])) + cC * m5[r];
      out[r] = h5[r] + dtg * Lm;
    }
#pragma unroll
    for (int r = 0; r < 2; r++) {
      ph3[r] = ph2[r];
      ph2[r] = ph1[r];
      ph1[r] = in[r];
      ux1[r] = inux[r];
      uy1[r] = inuy[r];
      uz2[r] = uz1[r];
      uz1[r] = inuz[r];
      h5[r] = h4[r];
      h4[r] = h3[r];
      h3[r] = h2[r];
      h2[r] = hnew[r];
      fh4[r] = fh3[r];
      fh3[r] = fh2[r];
      m6[r] = m5[r];
      m5[r] = m4[r];
      m4[r] = mnew[r];
      fm6[r] = fm5[r];
      fm5[r] = fm4[r];
    }
    const int zo = t - 5;
    if (zo >= z0 && zo < z1) {
      if (out0) phi_out[col0 + plane * zo] = out[0];
      if (out1) phi_out[col1 + plane * zo] = out[1];
    }
  };
  // unrolled by two so the queue slot and the parity are static
  for (int t = t0; t < t1; t += 2) {
    iterate(t, 0);
    if (t + 1 < t1) iterate(t + 1, 1);
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

// Drop statistics for Laplace's law (Sec. 2, Eq. surftens), stage 1: per
// block, in double and a fixed order, over the sites whose minimum-image
// distance from the centre (cx, cy, cz) is below r_in (inside) or above
// r_out (outside), the count and the sums of the bulk pressure of
// Eq. diagpress without gradient terms, p0 = n c_s^2 + a phi^2/2 + 3b phi^4/4,
// of phi and of n, and the sum of phi over all sites:
// part[blk*16 + k]: 0..3 count, p0, phi, n inside; 4..7 outside; 8 sum phi.
template <int K>
__device__ __forceinline__ void block_sum(double v[K], double *out) {
  __shared__ double red[4][K];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; k++) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; k++) red[wid][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; k++) out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
}

template <class L, typename T, int TX, int TY, int TZ>
__global__ void __launch_bounds__(256) k_drop_stats(KParams p, const T *__restrict__ gin, const T *__restrict__ phi,
                                                    double cx, double cy, double cz, double rin2, double rout2,
                                                    double *__restrict__ part) {
  constexpr int D = L::D;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = D == 3 ? blockIdx.z * TZ : 0;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const double a = p.a, b = p.b;
  auto image = [](double d, int n) { return d - n * floor(d / n + 0.5); };
  for (int s = threadIdx.x; s < TX * TY * TZ; s += blockDim.x) {
    const int tx = s % TX, ty = (s / TX) % TY, tz = s / (TX * TY);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    if (x >= p.nx || y >= p.ny || z >= p.nz) continue;
    T f[L::Q], dn, j[3];
    pull<L>(p, gin, x, y, z, f, dn, j);
    const double n = p.rho0 + double(dn);
    const double ph = double(phi[x + p.nx * (y + p.ny * z)]);
    const double dx = image(x - cx, p.nx), dy = image(y - cy, p.ny), dz = D == 3 ? image(z - cz, p.nz) : 0.0;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double p0 = n / 3.0 + 0.5 * a * ph * ph + 0.75 * b * ph * ph * ph * ph;
    acc[8] += ph;
    const int o = r2 < rin2 ? 0 : (r2 > rout2 ? 4 : -1);
    if (o >= 0) {
      acc[o] += 1.0;
      acc[o + 1] += p0;
      acc[o + 2] += ph;
      acc[o + 3] += n;
    }
  }
  const int blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  block_sum<9>(acc, part + (size_t)blk * 16);
}

// Stage 2 of the drop statistics: one block folds the partials in a fixed order.
__global__ void __launch_bounds__(256) k_drop_stats_final(int nblk, const double *__restrict__ part,
                                                          double *__restrict__ out) {
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < 9; k++) acc[k] += part[(size_t)b * 16 + k];
  block_sum<9>(acc, out);
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
