// Motion update around the force path: velocity Verlet (each MD iteration computes the
// forces on every atom, then updates the atoms' motion: Section 1, Section 2.1; the paper
// names no integrator). Positions, velocities and forces stay in HBM in the caller's order;
// one thread per atom. Units: A, fs, amu, kcal/mol.
#include "md_common.hpp"

namespace md {
namespace {

constexpr float kAccel = 4.184e-4f;    // (kcal/mol/A)/amu in A/fs^2
constexpr int kKeThreads = 256;

// v += h a; x += dt v, wrapped into [0, L) by one add or subtract of L (a step moves an
// atom far less than a box edge; one that moved farther stays outside and the force path
// flags it)
__global__ __launch_bounds__(256) void k_vv_kick_drift(int64_t n, float* __restrict__ pos,
                                                       float* __restrict__ vel,
                                                       const float* __restrict__ force,
                                                       const float* __restrict__ inv_mass,
                                                       float h, float dt, float L0, float L1,
                                                       float L2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float s = inv_mass[i] * kAccel;
  const float L[3] = {L0, L1, L2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float v = fmaf(h * s, force[3 * i + c], vel[3 * i + c]);
    float x = fmaf(dt, v, pos[3 * i + c]);
    if (x >= L[c]) x -= L[c];
    else if (x < 0.f) x += L[c];
    vel[3 * i + c] = v;
    pos[3 * i + c] = x;
  }
}

// v += h a, and this block's kinetic energy sum m v^2 / 2 (in amu A^2/fs^2, float64, one
// fixed tree order) into kpart[block]
__global__ __launch_bounds__(kKeThreads) void k_vv_kick(int64_t n, float* __restrict__ vel,
                                                        const float* __restrict__ force,
                                                        const float* __restrict__ inv_mass,
                                                        float h, double* __restrict__ kpart) {
  __shared__ double s_e[kKeThreads];
  const int64_t i = (int64_t)blockIdx.x * kKeThreads + threadIdx.x;
  double e = 0.0;
  if (i < n) {
    const float im = inv_mass[i];
    const float s = im * kAccel;
    double v2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float v = fmaf(h * s, force[3 * i + c], vel[3 * i + c]);
      vel[3 * i + c] = v;
      v2 += (double)v * (double)v;
    }
    e = im > 0.f ? 0.5 * v2 / (double)im : 0.0;   // a pinned atom (1/m = 0) does not move
  }
  s_e[threadIdx.x] = e;
  __syncthreads();
  for (int off = kKeThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s_e[threadIdx.x] += s_e[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) kpart[blockIdx.x] = s_e[0];
}

// the blocks' partials summed in a fixed order, in kcal/mol
__global__ __launch_bounds__(kKeThreads) void k_ke_sum(const double* __restrict__ kpart,
                                                       int64_t nb, double* __restrict__ ke) {
  __shared__ double s_e[kKeThreads];
  double e = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kKeThreads) e += kpart[b];
  s_e[threadIdx.x] = e;
  __syncthreads();
  for (int off = kKeThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s_e[threadIdx.x] += s_e[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *ke = s_e[0] / (double)kAccel;
}

}  // namespace

int64_t ke_blocks(int64_t n) { return n > 0 ? (n + kKeThreads - 1) / kKeThreads : 1; }

hipError_t launch_vv_kick_drift(int64_t n, float* pos, float* vel, const float* force,
                                const float* inv_mass, float h, float dt, const float* L,
                                hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_vv_kick_drift, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n,
                     pos, vel, force, inv_mass, h, dt, L[0], L[1], L[2]);
  return hipGetLastError();
}

hipError_t launch_vv_kick(int64_t n, float* vel, const float* force, const float* inv_mass,
                          float h, double* kpart, double* ke, hipStream_t stream) {
  const int64_t nb = n > 0 ? ke_blocks(n) : 0;
  if (nb > 0)
    hipLaunchKernelGGL(k_vv_kick, dim3((unsigned)nb), dim3(kKeThreads), 0, stream, n, vel, force,
                       inv_mass, h, kpart);
  hipLaunchKernelGGL(k_ke_sum, dim3(1), dim3(kKeThreads), 0, stream, kpart, nb, ke);
  return hipGetLastError();
}

}  // namespace md
