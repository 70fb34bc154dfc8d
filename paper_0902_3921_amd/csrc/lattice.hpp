// lattice.hpp -- velocity sets of the lattice Boltzmann step, as
// compile-time tables so that every population loop unrolls into code with
// constant velocities.
//
// D2Q9 is the lattice of Sec. 2.1 (Fig. 1): rest velocity, four axis links of
// length 1 and four diagonals of length sqrt(2), weights 4/9, 1/9, 1/36,
// c_s^2 = 1/3.  D3Q19 is its three-dimensional counterpart: rest 1/3, six
// faces 1/18, twelve edges 1/36.  The velocity order is part of the C ABI
// (documented in hlb.h).
#pragma once

#include <hip/hip_runtime.h>

namespace hlb {

struct D2Q9 {
  static constexpr int D = 2;
  static constexpr int Q = 9;
  __host__ __device__ static constexpr int e(int i, int k) {
    constexpr int E[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                             {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    return E[i][k];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  // index of the opposite velocity, e_opp(i) = -e_i
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int O[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    return O[i];
  }
};

struct D3Q19 {
  static constexpr int D = 3;
  static constexpr int Q = 19;
  __host__ __device__ static constexpr int e(int i, int k) {
    constexpr int E[19][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},   {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1}};
    return E[i][k];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  __host__ __device__ static constexpr int opp(int i) {
    return i == 0 ? 0 : (i % 2 == 1 ? i + 1 : i - 1);
  }
};

}  // namespace hlb
