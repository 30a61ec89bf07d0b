// D3Q19 kernels around the step: initial state, the strain query, canonical gather/scatter
// and the diagnostics reduction. One thread per node (the reduction: one x-row per block at
// a time).
#include <hip/hip_runtime.h>

#include "d3q19.h"
#include "d3q19_node.h"
#include "internal.h"
#include "launch.h"
#include "reduce.h"

namespace lbm {
namespace d3q19 {

// ------------------------------------------------------------------------------------------
// Strain of the current state (read only)
// ------------------------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(kMaxBlock) void strain_kernel(Geo G, ModelF M, ViscF V, ForceF Fo, const S* buf,
                                                     const float* snu_f, int kind, float* S_out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= G.nx || y >= G.ny) return;
  const Node<Q, S> nb = node_at<Q, S>(G, x, y, z);
  float g[Q];
  pull_rows<Lat, S>(buf, G, nb.rows, y, g);
  const Pairs P = make_pairs(g);
  const float drho = delta_rho(P);
  float jx = momentum<0>(P), jy = momentum<1>(P), jz = momentum<2>(P);
  float Fx, Fy, Fz;
  load_force(Fo, G.N, nb.self, Fx, Fy, Fz);
  jx += 0.5f * Fx;
  jy += 0.5f * Fy;
  jz += 0.5f * Fz;
  const Neq n = noneq_moments(P, drho, jx, jy, jz, M);
  const StrainIn<true> si = strain_in_state(n, jx, jy, jz, Fx, Fy, Fz, M, Fo);
  const float snu = V.kind == 3 ? implicit_rate(P, drho, jx, jy, jz, si, M, V) : (snu_f ? snu_f[nb.self] : M.s[9]);
  float S6[6];
  if (kind == 2) {
    float r[Q];
    rates_with(M, snu, r);
    strain_chai_in(P, drho, jx, jy, jz, r, si, M.inv_rho0, S6);
  } else {
    strain_yu(si.ns, M.s[1], snu, M.inv_rho0, S6);
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) stream_store(&S_out[static_cast<size_t>(c) * G.N + nb.self], S6[c]);
}

// ------------------------------------------------------------------------------------------
// Initial state g^eq(delta_rho, rho0 u) [+ Chapman-Enskog non-equilibrium part]
// ------------------------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(kMaxBlock) void init_kernel(Geo G, ModelF M, S* buf, float* snu, const float* rho_u,
                                                   const float* grad_u) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= G.nx || y >= G.ny) return;
  const Node<Q, S> nb = node_at<Q, S>(G, x, y, z);
  const unsigned self = nb.self;
  float drho = 0.f, ux = 0.f, uy = 0.f, uz = 0.f;
  if (rho_u) {
    drho = rho_u[self];
    ux = rho_u[G.N + self];
    uy = rho_u[2 * static_cast<size_t>(G.N) + self];
    uz = rho_u[3 * static_cast<size_t>(G.N) + self];
  }
  float g[Q];
  equilibrium(drho, M.rho0 * ux, M.rho0 * uy, M.rho0 * uz, M.inv_rho0, g);
  if (grad_u) {
    // d[a*3+b] = d j_b / d x_a; non-equilibrium moments of the Chapman-Enskog relations
    // (Eq. YuLuobasis), every other row zero.
    float d[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) d[k] = M.rho0 * grad_u[static_cast<size_t>(k) * G.N + self];
    const float div = d[0] + d[4] + d[8];
    const float s1 = M.s[1], sn = M.s[9];
    float mn[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) mn[k] = 0.0f;
    mn[1] = -38.0f * div / (3.0f * s1);
    mn[9] = -2.0f * (3.0f * d[0] - div) / (3.0f * sn);
    mn[11] = -2.0f * (d[4] - d[8]) / (3.0f * sn);
    mn[13] = -(d[1] + d[3]) / (3.0f * sn);
    mn[14] = -(d[5] + d[7]) / (3.0f * sn);
    mn[15] = -(d[2] + d[6]) / (3.0f * sn);
    add_neq_from_moments(mn, g);
  }
  scatter_rows<Lat, S>(buf, G, nb.rows, y, g);
  if (snu) snu[self] = M.s[9];
}

template <typename S>
__global__ __launch_bounds__(kMaxBlock) void get_kernel(Geo G, const S* buf, float* canon) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= G.nx || y >= G.ny) return;
  const Node<Q, S> nb = node_at<Q, S>(G, x, y, z);
  float g[Q];
  pull_rows<Lat, S>(buf, G, nb.rows, y, g);
  store_local<Q>(canon, G, nb.self * 4u, g);
}

template <typename S>
__global__ __launch_bounds__(kMaxBlock) void set_kernel(Geo G, S* buf, const float* canon) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= G.nx || y >= G.ny) return;
  const Node<Q, S> nb = node_at<Q, S>(G, x, y, z);
  float g[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) g[i] = canon[static_cast<size_t>(i) * G.N + nb.self];
  scatter_rows<Lat, S>(buf, G, nb.rows, y, g);
}

// ------------------------------------------------------------------------------------------
// Diagnostics: mass, momentum, kinetic energy, sum S:S (Yu), max |u|, non-finite count
// ------------------------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(256) void reduce_kernel(Geo G, ModelF M, ViscF V, ForceF Fo, const S* buf,
                                                     const float* snu_f, double* partials) {
  double acc[kReduceVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  // blocks take whole x-rows in turn; the threads of a block walk along the row
  const unsigned rows = static_cast<unsigned>(G.ny) * G.nz;
  for (unsigned r = blockIdx.x; r < rows; r += gridDim.x) {
    const int y = r % G.ny;
    const int z = r / G.ny;
    for (int x = threadIdx.x; x < G.nx; x += blockDim.x) {
      const Node<Q, S> nb = node_at<Q, S>(G, x, y, z);
      float g[Q];
      pull_rows<Lat, S>(buf, G, nb.rows, y, g);
      int bad = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) bad += !isfinite(g[i]);
      const Pairs P = make_pairs(g);
      const float drho = delta_rho(P);
      float jx = momentum<0>(P), jy = momentum<1>(P), jz = momentum<2>(P);
      float Fx, Fy, Fz;
      load_force(Fo, G.N, nb.self, Fx, Fy, Fz);
      jx += 0.5f * Fx;
      jy += 0.5f * Fy;
      jz += 0.5f * Fz;
      const Neq n = noneq_moments(P, drho, jx, jy, jz, M);
      const StrainIn<true> si = strain_in_state(n, jx, jy, jz, Fx, Fy, Fz, M, Fo);
      const float snu = V.kind == 3 ? implicit_rate(P, drho, jx, jy, jz, si, M, V) : (snu_f ? snu_f[nb.self] : M.s[9]);
      float S6[6];
      strain_yu(si.ns, M.s[1], snu, M.inv_rho0, S6);
      const double jj = static_cast<double>(jx) * jx + static_cast<double>(jy) * jy + static_cast<double>(jz) * jz;
      acc[0] += drho;
      acc[1] += jx;
      acc[2] += jy;
      acc[3] += jz;
      acc[4] += jj * (0.5 / M.rho0);
      double ss = 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) ss += (c < 3 ? 1.0 : 2.0) * static_cast<double>(S6[c]) * S6[c];
      acc[5] += ss;
      acc[6] = fmax(acc[6], jj);  // max |j|^2: the final pass takes sqrt(.) / rho0 once
      acc[7] += bad;
    }
  }
  block_reduce_store(acc, partials);
}

// ------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------
template <typename S>
static const S* cbuf(const void* p) {
  return static_cast<const S*>(p);
}

hipError_t launch_strain(int storage, const Geo& G, const ModelF& M, const ViscF& V, const ForceF& Fo, const void* buf,
                         const float* snu, int kind, float* S_out, hipStream_t st) {
  const Launch L = node_launch(G);
  // whole 256-node rows: 5 blocks per CU instead of 8 (+1.9 % at 256^3; 4 blocks lost 0.6 %)
  const size_t lds = (L.block.x == 256 && L.block.y == 1) ? lds_cap_bytes(5, 0) : 0;
  switch (storage) {
    case 0: hipLaunchKernelGGL(strain_kernel<float>, L.grid, L.block, lds, st, G, M, V, Fo, cbuf<float>(buf), snu, kind, S_out); break;
    case 1: hipLaunchKernelGGL(strain_kernel<_Float16>, L.grid, L.block, 0, st, G, M, V, Fo, cbuf<_Float16>(buf), snu, kind, S_out); break;
    case 2: hipLaunchKernelGGL(strain_kernel<__bf16>, L.grid, L.block, 0, st, G, M, V, Fo, cbuf<__bf16>(buf), snu, kind, S_out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_init(int storage, const Geo& G, const ModelF& M, void* buf, float* snu, const float* rho_u,
                       const float* grad_u, hipStream_t st) {
  const Launch L = node_launch(G);
  switch (storage) {
    case 0: hipLaunchKernelGGL(init_kernel<float>, L.grid, L.block, 0, st, G, M, static_cast<float*>(buf), snu, rho_u, grad_u); break;
    case 1: hipLaunchKernelGGL(init_kernel<_Float16>, L.grid, L.block, 0, st, G, M, static_cast<_Float16*>(buf), snu, rho_u, grad_u); break;
    case 2: hipLaunchKernelGGL(init_kernel<__bf16>, L.grid, L.block, 0, st, G, M, static_cast<__bf16*>(buf), snu, rho_u, grad_u); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_get(int storage, const Geo& G, const void* buf, float* canon, hipStream_t st) {
  const Launch L = node_launch(G);
  switch (storage) {
    case 0: hipLaunchKernelGGL(get_kernel<float>, L.grid, L.block, 0, st, G, cbuf<float>(buf), canon); break;
    case 1: hipLaunchKernelGGL(get_kernel<_Float16>, L.grid, L.block, 0, st, G, cbuf<_Float16>(buf), canon); break;
    case 2: hipLaunchKernelGGL(get_kernel<__bf16>, L.grid, L.block, 0, st, G, cbuf<__bf16>(buf), canon); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_set(int storage, const Geo& G, void* buf, const float* canon, hipStream_t st) {
  const Launch L = node_launch(G);
  switch (storage) {
    case 0: hipLaunchKernelGGL(set_kernel<float>, L.grid, L.block, 0, st, G, static_cast<float*>(buf), canon); break;
    case 1: hipLaunchKernelGGL(set_kernel<_Float16>, L.grid, L.block, 0, st, G, static_cast<_Float16*>(buf), canon); break;
    case 2: hipLaunchKernelGGL(set_kernel<__bf16>, L.grid, L.block, 0, st, G, static_cast<__bf16*>(buf), canon); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(int storage, const Geo& G, const ModelF& M, const ViscF& V, const ForceF& Fo, const void* buf,
                         const float* snu, double* partials, double* out, hipStream_t st) {
  unsigned nb = static_cast<unsigned>(G.ny) * G.nz;  // one x-row per block at a time
  if (nb > static_cast<unsigned>(kReduceBlocks)) nb = kReduceBlocks;
  // FP32: 4 blocks per CU instead of the 5 its registers allow (3.5 % less time per call at
  // 256^3; 3 blocks 7 % more)
  const size_t lds = lds_cap_bytes(4, 4 * kReduceVals * sizeof(double));
  switch (storage) {
    case 0: hipLaunchKernelGGL(reduce_kernel<float>, dim3(nb), dim3(256), lds, st, G, M, V, Fo, cbuf<float>(buf), snu, partials); break;
    case 1: hipLaunchKernelGGL(reduce_kernel<_Float16>, dim3(nb), dim3(256), 0, st, G, M, V, Fo, cbuf<_Float16>(buf), snu, partials); break;
    case 2: hipLaunchKernelGGL(reduce_kernel<__bf16>, dim3(nb), dim3(256), 0, st, G, M, V, Fo, cbuf<__bf16>(buf), snu, partials); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_final(partials, static_cast<int>(nb), out, st, static_cast<double>(M.rho0));
}

}  // namespace d3q19
}  // namespace lbm
