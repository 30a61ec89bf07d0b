// D3Q15 kernels: the fused pull-stream / collide / strain step on the fifteen-velocity
// lattice (the Chai formula of Section 5.3 and the Yu-type formula of Section 5.4), plus
// initial state, strain query, canonical gather/scatter and the diagnostics reduction.
// One thread per node, the launch shape and memory layout of the D3Q19 path.
#include <hip/hip_runtime.h>

#include "d3q15.h"
#include "internal.h"
#include "launch.h"
#include "reduce.h"

namespace lbm {
namespace d3q15 {

__device__ __forceinline__ void load_force(const ForceF& Fo, unsigned N, unsigned self, float& Fx, float& Fy,
                                           float& Fz) {
  if (Fo.mode == 1) {
    Fx = Fo.F[0];
    Fy = Fo.F[1];
    Fz = Fo.F[2];
  } else if (Fo.mode == 2) {
    Fx = Fo.field[self];
    Fy = Fo.field[N + self];
    Fz = Fo.field[2 * static_cast<size_t>(N) + self];
  } else {
    Fx = Fy = Fz = 0.0f;
  }
}

__device__ __forceinline__ void rates_with(const ModelF& M, float snu, float (&r)[Q]) {
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    r[k] = is_nu_slot(k) ? snu : M.s[k];
  });
}

__device__ __forceinline__ float strain_sq(const float (&S)[6]) {
  return S[0] * S[0] + S[1] * S[1] + S[2] * S[2] + 2.0f * (S[3] * S[3] + S[4] * S[4] + S[5] * S[5]);
}

// The force-corrected strain (optional) takes the non-equilibrium part plus half the Guo
// source, m - m^eq + S_F/2. StrainIn holds the moments the Yu-type formula reads (ns) and,
// with CORR, h = S_F/2, which the Chai formula adds as the Yu-type contraction of h with the
// same rates (the Chai contraction of F-bar/2 in moment space). Without CORR only the plain
// moments are held.
template <bool CORR>
struct StrainIn {
  Neq ns;
  Neq h;
};

template <bool CORR>
__device__ __forceinline__ StrainIn<CORR> strain_in(const Neq& n, const float (&SF)[Q]) {
  StrainIn<CORR> si;
  if constexpr (CORR) {
    static_for<Q>([&](auto ki) {
      constexpr int k = ki;
      si.h.m[k] = 0.5f * SF[k];
      si.ns.m[k] = n.m[k] + si.h.m[k];
    });
  } else {
    si.ns = n;
  }
  return si;
}

// The read-only kernels take the corrected form always, with a zero source when the
// correction is off.
__device__ __forceinline__ StrainIn<true> strain_in_state(const Neq& n, float jx, float jy, float jz, float Fx, float Fy, float Fz,
                                                          const ModelF& M, const ForceF& Fo) {
  float SF[Q];
  if (Fo.strain_corr) {
    force_moments(jx, jy, jz, Fx, Fy, Fz, M.inv_rho0, SF);
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) SF[k] = 0.0f;
  }
  return strain_in<true>(n, SF);
}

template <bool CORR>
__device__ __forceinline__ void strain_chai_in(const Pairs& P, float drho, float jx, float jy, float jz, const float (&rates)[Q],
                                               const StrainIn<CORR>& si, float inv_rho0, float (&S)[6]) {
  strain_chai(P, drho, jx, jy, jz, rates, inv_rho0, S);
  if constexpr (CORR) {
    float Sh[6];
    strain_yu(si.h, rates[1], rates[9], inv_rho0, Sh);
#pragma unroll
    for (int c = 0; c < 6; ++c) S[c] += Sh[c];
  }
}

// s_nu of the implicit Smagorinsky coupling at one node, from the formula V selects (both
// are affine in s_nu: split into the part at the other rates and the s_nu rows).
template <bool CORR>
__device__ __forceinline__ float implicit_rate(const Pairs& P_, float drho, float jx, float jy, float jz,
                                               const StrainIn<CORR>& si, const ModelF& M, const ViscF& V) {
  float P[6], A[6];
  if (V.drive_chai) {
    float rb[Q], rn[Q];
    rates_with(M, 0.0f, rb);
    static_for<Q>([&](auto ki) {
      constexpr int k = ki;
      rn[k] = is_nu_slot(k) ? 1.0f : 0.0f;
    });
    strain_chai_in(P_, drho, jx, jy, jz, rb, si, M.inv_rho0, P);
    strain_chai_in(P_, drho, jx, jy, jz, rn, si, M.inv_rho0, A);
  } else {
    strain_yu(si.ns, M.s[1], 0.0f, M.inv_rho0, P);
    strain_yu(si.ns, 0.0f, 1.0f, M.inv_rho0, A);
  }
  return implicit_smagorinsky(P, A, V.nu0, V.csmag2);
}

// The s_nu a strain query or the diagnostics take the strain with: the stored lagged rate,
// the implicit rate of the state itself, or the constant rate.
__device__ __forceinline__ float query_rate(const Pairs& P, float drho, float jx, float jy, float jz, const StrainIn<true>& si,
                                            const ModelF& M, const ViscF& V, const float* snu_f, unsigned self) {
  if (V.kind == 3) return implicit_rate(P, drho, jx, jy, jz, si, M, V);
  return snu_f ? snu_f[self] : M.s[9];
}

// XMODE: how a block pulls along x (pull_mode: 0 part rows, 1 whole rows, 2 whole rows with
// the LDS exchange). CORR: the force-corrected strain (a separate instance, so that the plain
// step keeps its register budget).
template <typename S, bool WALLS, int XMODE, bool CORR>
__global__ __launch_bounds__(kMaxBlock) void step_kernel(Geo G, ModelF M, ViscF V, ForceF Fo, StepIO io) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= G.nx || y >= G.ny) return;
  const unsigned self = node_index(G, x, y, z);
  const Rows<Q, S> r = rows_of<Q, S>(G, x, y, z);
  float g[Q];
  if constexpr (XMODE == 2) pull_rows_staged<Lat, S, WALLS>(static_cast<const S*>(io.src), G, r, y, g);
  else pull_rows<Lat, S, WALLS, XMODE == 1>(static_cast<const S*>(io.src), G, r, y, g);
  const Pairs P = make_pairs(g);
  const float drho = delta_rho(P);
  float jx = momentum<0>(P), jy = momentum<1>(P), jz = momentum<2>(P);
  float Fx, Fy, Fz;
  load_force(Fo, G.N, self, Fx, Fy, Fz);
  if (Fo.mode) {
    jx = __builtin_fmaf(0.5f, Fx, jx);
    jy = __builtin_fmaf(0.5f, Fy, jy);
    jz = __builtin_fmaf(0.5f, Fz, jz);
  }
  const Neq n = noneq_moments(P, drho, jx, jy, jz, M.inv_rho0);
  // the Guo source in moment space; with CORR formed before the strain (half of it joins the
  // non-equilibrium part the strain takes)
  float SF[Q];
  if constexpr (CORR) force_moments(jx, jy, jz, Fx, Fy, Fz, M.inv_rho0, SF);
  const StrainIn<CORR> si = strain_in<CORR>(n, SF);
  float Syu[6], Sch[6];
  float snu = M.s[9];
  if (V.kind == 3) {
    // implicit coupling: the strain at the rate of this very collision
    snu = implicit_rate(P, drho, jx, jy, jz, si, M, V);
    if (io.S_out) {
      if (io.emit == 2) {
        float r[Q];
        rates_with(M, snu, r);
        strain_chai_in(P, drho, jx, jy, jz, r, si, M.inv_rho0, Sch);
      } else {
        strain_yu(si.ns, M.s[1], snu, M.inv_rho0, Syu);
      }
#pragma unroll
      for (int c = 0; c < 6; ++c)
        stream_store(&io.S_out[static_cast<size_t>(c) * G.N + self], io.emit == 2 ? Sch[c] : Syu[c]);
    }
  } else {
    // lagged coupling: the strain of the incoming state with the rates of the previous collision
    const float snu_prev = io.snu ? io.snu[self] : M.s[9];
    const bool need_yu = io.emit == 1 || (V.kind != 0 && !V.drive_chai);
    const bool need_chai = io.emit == 2 || (V.kind != 0 && V.drive_chai);
    if (need_yu) strain_yu(si.ns, M.s[1], snu_prev, M.inv_rho0, Syu);
    if (need_chai) {
      float r[Q];
      rates_with(M, snu_prev, r);
      strain_chai_in(P, drho, jx, jy, jz, r, si, M.inv_rho0, Sch);
    }
    if (io.S_out) {
#pragma unroll
      for (int c = 0; c < 6; ++c)
        stream_store(&io.S_out[static_cast<size_t>(c) * G.N + self], io.emit == 2 ? Sch[c] : Syu[c]);
    }
    if (V.kind != 0) {
      snu = viscous_rate(V.drive_chai ? strain_sq(Sch) : strain_sq(Syu), V);
      io.snu[self] = snu;
    }
  }
  // relaxation in moment space with the Guo term, then the back-transform
  float dm[Q];
  dm[0] = 0.0f;
  dm[3] = Fx;
  dm[5] = Fy;
  dm[7] = Fz;
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    if constexpr (k != 0 && k != 3 && k != 5 && k != 7) dm[k] = -(is_nu_slot(k) ? snu : M.s[k]) * n.m[k];
  });
  if (Fo.mode) {
    if constexpr (!CORR) force_moments(jx, jy, jz, Fx, Fy, Fz, M.inv_rho0, SF);
    static_for<Q>([&](auto ki) {
      constexpr int k = ki;
      if constexpr (k != 0 && k != 3 && k != 5 && k != 7 && k != 14) {
        const float sk = is_nu_slot(k) ? snu : M.s[k];
        dm[k] = __builtin_fmaf(1.0f - 0.5f * sk, SF[k], dm[k]);
      }
    });
  }
  add_back_transform(dm, g);
  store_rows<Q>(static_cast<S*>(io.dst), G, r, g);
}

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
  float Fx, Fy, Fz;
  load_force(Fo, G.N, nb.self, Fx, Fy, Fz);
  const float jx = momentum<0>(P) + 0.5f * Fx, jy = momentum<1>(P) + 0.5f * Fy, jz = momentum<2>(P) + 0.5f * Fz;
  const Neq n = noneq_moments(P, drho, jx, jy, jz, M.inv_rho0);
  const StrainIn<true> si = strain_in_state(n, jx, jy, jz, Fx, Fy, Fz, M, Fo);
  const float snu = query_rate(P, drho, jx, jy, jz, si, M, V, snu_f, nb.self);
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

template <typename S>
__global__ __launch_bounds__(kMaxBlock) void init_kernel(Geo G, ModelF M, S* buf, float* snu, const float* rho_u,
                                                         const float* grad_u) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= G.nx || y >= G.ny) return;
  const Node<Q, S> nb = node_at<Q, S>(G, x, y, z);
  const unsigned self = nb.self;
  const size_t N = G.N;
  float drho = 0.f, ux = 0.f, uy = 0.f, uz = 0.f;
  if (rho_u) {
    drho = rho_u[self];
    ux = rho_u[N + self];
    uy = rho_u[2 * N + self];
    uz = rho_u[3 * N + self];
  }
  float g[Q];
  equilibrium(drho, M.rho0 * ux, M.rho0 * uy, M.rho0 * uz, M.inv_rho0, g);
  if (grad_u) {
    // d[a*3+b] = d j_b / d x_a; the non-equilibrium moments that invert the Yu-type formula
    float d[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) d[k] = M.rho0 * grad_u[static_cast<size_t>(k) * N + self];
    const float div = d[0] + d[4] + d[8];
    const float sn = M.s[9];
    float mn[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) mn[k] = 0.0f;
    mn[1] = -2.0f * div / (3.0f * M.s[1]);
    mn[9] = -2.0f * (3.0f * d[0] - div) / (3.0f * sn);
    mn[10] = -2.0f * (d[4] - d[8]) / (3.0f * sn);
    mn[11] = -(d[1] + d[3]) / (3.0f * sn);
    mn[12] = -(d[5] + d[7]) / (3.0f * sn);
    mn[13] = -(d[2] + d[6]) / (3.0f * sn);
    add_back_transform(mn, g);
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
      float Fx, Fy, Fz;
      load_force(Fo, G.N, nb.self, Fx, Fy, Fz);
      const float jx = momentum<0>(P) + 0.5f * Fx, jy = momentum<1>(P) + 0.5f * Fy, jz = momentum<2>(P) + 0.5f * Fz;
      const Neq n = noneq_moments(P, drho, jx, jy, jz, M.inv_rho0);
      float S6[6];
      const StrainIn<true> si = strain_in_state(n, jx, jy, jz, Fx, Fy, Fz, M, Fo);
      strain_yu(si.ns, M.s[1], query_rate(P, drho, jx, jy, jz, si, M, V, snu_f, nb.self), M.inv_rho0, S6);
      const double jj = static_cast<double>(jx) * jx + static_cast<double>(jy) * jy + static_cast<double>(jz) * jz;
      acc[0] += drho;
      acc[1] += jx;
      acc[2] += jy;
      acc[3] += jz;
      acc[4] += jj * (0.5 / M.rho0);
      acc[5] += static_cast<double>(S6[0]) * S6[0] + static_cast<double>(S6[1]) * S6[1] +
                static_cast<double>(S6[2]) * S6[2] +
                2.0 * (static_cast<double>(S6[3]) * S6[3] + static_cast<double>(S6[4]) * S6[4] +
                       static_cast<double>(S6[5]) * S6[5]);
      acc[6] = fmax(acc[6], jj);  // max |j|^2: the final pass takes sqrt(.) / rho0 once
      acc[7] += bad;
    }
  }
  block_reduce_store(acc, partials);
}

template <typename S>
static const S* cb(const void* p) {
  return static_cast<const S*>(p);
}

template <typename S, bool CORR>
static void launch_step_c(bool walls, const Launch& L, hipStream_t st, const Geo& G, const ModelF& M, const ViscF& V,
                          const ForceF& Fo, const StepIO& io) {
  const int mode = pull_mode(G, L.block);
  // FP32 in whole 256-node rows: 4 blocks per CU instead of 7 (+4.4 % at 256^3; 3 blocks lost
  // 2 %). See lds_cap_bytes.
  size_t lds = 0;
  if constexpr (sizeof(S) == 4) {
    if (mode == 2 && L.block.x == 256 && L.block.y == 1) lds = lds_cap_bytes(4, staged_lds_bytes<Lat>());
  }
  switch (mode + (walls ? 3 : 0)) {
    case 0: hipLaunchKernelGGL((step_kernel<S, false, 0, CORR>), L.grid, L.block, lds, st, G, M, V, Fo, io); break;
    case 1: hipLaunchKernelGGL((step_kernel<S, false, 1, CORR>), L.grid, L.block, lds, st, G, M, V, Fo, io); break;
    case 2: hipLaunchKernelGGL((step_kernel<S, false, 2, CORR>), L.grid, L.block, lds, st, G, M, V, Fo, io); break;
    case 3: hipLaunchKernelGGL((step_kernel<S, true, 0, CORR>), L.grid, L.block, lds, st, G, M, V, Fo, io); break;
    case 4: hipLaunchKernelGGL((step_kernel<S, true, 1, CORR>), L.grid, L.block, lds, st, G, M, V, Fo, io); break;
    default: hipLaunchKernelGGL((step_kernel<S, true, 2, CORR>), L.grid, L.block, lds, st, G, M, V, Fo, io); break;
  }
}

template <typename S>
static void launch_step_t(bool walls, const Launch& L, hipStream_t st, const Geo& G, const ModelF& M, const ViscF& V,
                          const ForceF& Fo, const StepIO& io) {
  if (Fo.strain_corr) launch_step_c<S, true>(walls, L, st, G, M, V, Fo, io);
  else launch_step_c<S, false>(walls, L, st, G, M, V, Fo, io);
}

hipError_t launch_step(int storage, const Geo& G, const ModelF& M, const ViscF& V, const ForceF& Fo, const StepIO& io,
                       hipStream_t st) {
  const Launch L = node_launch(G);
  switch (storage) {
    case 0: launch_step_t<float>(G.walls != 0, L, st, G, M, V, Fo, io); break;
    case 1: launch_step_t<_Float16>(G.walls != 0, L, st, G, M, V, Fo, io); break;
    case 2: launch_step_t<__bf16>(G.walls != 0, L, st, G, M, V, Fo, io); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_strain(int storage, const Geo& G, const ModelF& M, const ViscF& V, const ForceF& Fo, const void* buf,
                         const float* snu, int kind, float* S_out, hipStream_t st) {
  const Launch L = node_launch(G);
  switch (storage) {
    case 0: hipLaunchKernelGGL(strain_kernel<float>, L.grid, L.block, 0, st, G, M, V, Fo, cb<float>(buf), snu, kind, S_out); break;
    case 1: hipLaunchKernelGGL(strain_kernel<_Float16>, L.grid, L.block, 0, st, G, M, V, Fo, cb<_Float16>(buf), snu, kind, S_out); break;
    case 2: hipLaunchKernelGGL(strain_kernel<__bf16>, L.grid, L.block, 0, st, G, M, V, Fo, cb<__bf16>(buf), snu, kind, S_out); break;
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
    case 0: hipLaunchKernelGGL(get_kernel<float>, L.grid, L.block, 0, st, G, cb<float>(buf), canon); break;
    case 1: hipLaunchKernelGGL(get_kernel<_Float16>, L.grid, L.block, 0, st, G, cb<_Float16>(buf), canon); break;
    case 2: hipLaunchKernelGGL(get_kernel<__bf16>, L.grid, L.block, 0, st, G, cb<__bf16>(buf), canon); break;
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

hipError_t launch_reduce(int storage, const Geo& G, const ModelF& M, const ViscF& V, const ForceF& Fo,
                         const void* buf, const float* snu, double* partials, double* out, hipStream_t st) {
  unsigned nb = static_cast<unsigned>(G.ny) * G.nz;  // one x-row per block at a time
  if (nb > static_cast<unsigned>(kReduceBlocks)) nb = kReduceBlocks;
  switch (storage) {
    case 0: hipLaunchKernelGGL(reduce_kernel<float>, dim3(nb), dim3(256), 0, st, G, M, V, Fo, cb<float>(buf), snu, partials); break;
    case 1: hipLaunchKernelGGL(reduce_kernel<_Float16>, dim3(nb), dim3(256), 0, st, G, M, V, Fo, cb<_Float16>(buf), snu, partials); break;
    case 2: hipLaunchKernelGGL(reduce_kernel<__bf16>, dim3(nb), dim3(256), 0, st, G, M, V, Fo, cb<__bf16>(buf), snu, partials); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_final(partials, static_cast<int>(nb), out, st, static_cast<double>(M.rho0));
}

}  // namespace d3q15
}  // namespace lbm
