// Discrete adjoint of the D3Q19 step (constant viscosity) and of the strain-squared loss.
//
// Forward step: g^{n+1} = P C(g^n, F), with the collision of Eq. mrteqvT written in moment
// space, m* = m - L (m - m^eq(drho, j)) + (I - L/2) S_F(j, F), j = (m_3, m_5, m_7) + F/2,
// g* = T^-1 m*, L = diag(s), and P the pull streaming. Its transpose, per node x:
//   lam~_i(x) = lam_i(x + c_i)          (P^T: a pull along -c_i, with the transpose of
//                                         bounce-back at y-walls)
//   mu       = D^-1 T lam~               (T^-T = D^-1 T, rows of T orthogonal)
//   nu       = (dm*/dm)^T mu,  dm*/dm = I - L + L E + (I - L/2) dS_F/dm
//   lam'(x)  = T^T nu
//   grad_F(x) += (dm*/dF)^T mu,  dm*/dF = L (dm^eq/dj)/2 + (I - L/2)(G(j) + (dS_F/dj)/2)
// E = dm^eq/dm has non-zero columns 0 (d/d drho) and 3, 5, 7 (d/dj); G(j) = dS_F/dF.
// All derivative rows are written from Eq. meq (rows 9..12 as in Eq. solvem) and from the
// Guo moments of the He-Luo equilibrium.
#include <hip/hip_runtime.h>

#include "d3q19.h"
#include "internal.h"
#include "reduce.h"

namespace lbm {
namespace d3q19 {

// Streaming transpose as a pull along -c.
struct LatRev {
  static constexpr int Q = 19;
  static constexpr int cx(int i) { return -CX[i]; }
  static constexpr int cy(int i) { return -CY[i]; }
  static constexpr int cz(int i) { return -CZ[i]; }
  static constexpr int opp(int i) { return DV.opp[i]; }
};

// Pull streaming (forward direction), for reading the internal post-collision state.
struct LatFwd {
  static constexpr int Q = 19;
  static constexpr int cx(int i) { return CX[i]; }
  static constexpr int cy(int i) { return CY[i]; }
  static constexpr int cz(int i) { return CZ[i]; }
  static constexpr int opp(int i) { return DV.opp[i]; }
};

// out_i = sum_k T_ki v_k (T^T v) with the pair parity of T.
__device__ __forceinline__ void apply_transpose(const float (&v)[Q], float (&out)[Q]) {
  float r0 = -0.0f;
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    if constexpr (DV.even[k]) r0 = acc_int<TM[k][0]>(r0, v[k]);
  });
  out[0] = r0;
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    constexpr int a = DV.pa[p];
    constexpr int b = DV.pb[p];
    float e = -0.0f, o = -0.0f;
    static_for<Q>([&](auto ki) {
      constexpr int k = ki;
      if constexpr (DV.even[k]) e = acc_int<TM[k][a]>(e, v[k]);
      else o = acc_int<TM[k][a]>(o, v[k]);
    });
    out[a] = e + o;
    out[b] = e - o;
  });
}

__device__ __forceinline__ void force_at(const ForceF& Fo, unsigned N, unsigned self, float& Fx, float& Fy, float& Fz) {
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

__global__ __launch_bounds__(kMaxBlock) void adjoint_kernel(Geo G, ModelF M, ForceF Fo, const float* __restrict__ j_n,
                                                      const float* __restrict__ lam_in, float* __restrict__ lam_out,
                                                      float* __restrict__ grad_force) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= G.nx || y >= G.ny) return;
  const Nbr ne = neighbours(G, x, y, z);
  const unsigned self = ne.self;
  const Nbr nb = in_bytes<float>(ne);

  float lt[Q];
  pull<LatRev, float>(lam_in, G, nb, y, lt);

  // mu = D^-1 T lam~
  const Pairs P = make_pairs(lt);
  float mu[Q];
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    mu[k] = moment<k>(P) * (1.0f / static_cast<float>(DV.D[k]));
  });

  const float jx = j_n[self], jy = j_n[G.N + self], jz = j_n[2 * static_cast<size_t>(G.N) + self];
  const float ir = M.inv_rho0;
  float w[Q], v[Q], nu[Q];
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    const float sk = M.s[k];
    w[k] = sk * mu[k];
    v[k] = (1.0f - 0.5f * sk) * mu[k];
    nu[k] = mu[k] - w[k];
  });
  // column 0 of E: d m^eq / d drho = (1, -11, omega_eps, 0, ...)
  nu[0] += w[0] - 11.0f * w[1] + M.om_eps * w[2];
  // columns 3, 5, 7 of E: d m^eq / d j
  const float e2 = 2.0f * M.om_epsj, oxx = M.om_xx;
  const float Ax = (38.0f * jx * w[1] + e2 * jx * w[2] + 4.0f * jx * w[9] + 4.0f * oxx * jx * w[10] + jy * w[13] +
                    jz * w[15]) * ir + w[3] - (2.0f / 3.0f) * w[4];
  const float Ay = (38.0f * jy * w[1] + e2 * jy * w[2] - 2.0f * jy * w[9] - 2.0f * oxx * jy * w[10] +
                    2.0f * jy * w[11] + 2.0f * oxx * jy * w[12] + jx * w[13] + jz * w[14]) * ir + w[5] -
                   (2.0f / 3.0f) * w[6];
  const float Az = (38.0f * jz * w[1] + e2 * jz * w[2] - 2.0f * jz * w[9] - 2.0f * oxx * jz * w[10] -
                    2.0f * jz * w[11] - 2.0f * oxx * jz * w[12] + jy * w[14] + jx * w[15]) * ir + w[7] -
                   (2.0f / 3.0f) * w[8];
  float Bx = 0.f, By = 0.f, Bz = 0.f, Fx = 0.f, Fy = 0.f, Fz = 0.f;
  if (Fo.mode) {
    force_at(Fo, G.N, self, Fx, Fy, Fz);
    // d S_F / d j (S_F = T F-bar, Guo moments of the He-Luo equilibrium)
    Bx = (38.0f * Fx * v[1] - 11.0f * Fx * v[2] + 4.0f * Fx * v[9] - 2.0f * Fx * v[10] + Fy * v[13] + Fz * v[15]) * ir;
    By = (38.0f * Fy * v[1] - 11.0f * Fy * v[2] - 2.0f * Fy * v[9] + Fy * v[10] + 2.0f * Fy * v[11] - Fy * v[12] +
          Fx * v[13] + Fz * v[14]) * ir;
    Bz = (38.0f * Fz * v[1] - 11.0f * Fz * v[2] - 2.0f * Fz * v[9] + Fz * v[10] - 2.0f * Fz * v[11] + Fz * v[12] +
          Fy * v[14] + Fx * v[15]) * ir;
  }
  nu[3] += Ax + Bx;
  nu[5] += Ay + By;
  nu[7] += Az + Bz;

  float lo[Q];
  apply_transpose(nu, lo);
  store_local<Q>(lam_out, G, nb.self, lo);

  if (grad_force) {
    // G(j) = d S_F / d F
    const float Cx = (38.0f * jx * v[1] - 11.0f * jx * v[2] + 4.0f * jx * v[9] - 2.0f * jx * v[10] + jy * v[13] +
                      jz * v[15]) * ir + v[3] - (2.0f / 3.0f) * v[4];
    const float Cy = (38.0f * jy * v[1] - 11.0f * jy * v[2] - 2.0f * jy * v[9] + jy * v[10] + 2.0f * jy * v[11] -
                      jy * v[12] + jx * v[13] + jz * v[14]) * ir + v[5] - (2.0f / 3.0f) * v[6];
    const float Cz = (38.0f * jz * v[1] - 11.0f * jz * v[2] - 2.0f * jz * v[9] + jz * v[10] - 2.0f * jz * v[11] +
                      jz * v[12] + jy * v[14] + jx * v[15]) * ir + v[7] - (2.0f / 3.0f) * v[8];
    grad_force[self] += 0.5f * (Ax + Bx) + Cx;
    grad_force[G.N + self] += 0.5f * (Ay + By) + Cy;
    grad_force[2 * static_cast<size_t>(G.N) + self] += 0.5f * (Az + Bz) + Cz;
  }
}

// Loss J = sum_x S:S (Yu strain of the current pre-collision state) and its gradients.
template <typename S>
__global__ __launch_bounds__(256) void loss_seed_kernel(Geo G, ModelF M, ForceF Fo, const S* __restrict__ buf,
                                                        float* __restrict__ lam_out, float* __restrict__ grad_force,
                                                        double* __restrict__ partials) {
  double acc[kReduceVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  const unsigned stride = gridDim.x * blockDim.x;
  for (unsigned idx = blockIdx.x * blockDim.x + threadIdx.x; idx < G.N; idx += stride) {
    const int x = idx % G.nx;
    const unsigned t = idx / G.nx;
    const int y = t % G.ny;
    const int z = t / G.ny;
    const Nbr nb = neighbours(G, x, y, z);
    const unsigned self = nb.self;
    float g[Q];
    pull<LatFwd, S>(buf, G, in_bytes<S>(nb), y, g);
    const Pairs P = make_pairs(g);
    const float drho = delta_rho(P);
    float Fx, Fy, Fz;
    force_at(Fo, G.N, self, Fx, Fy, Fz);
    const float jx = momentum<0>(P) + 0.5f * Fx, jy = momentum<1>(P) + 0.5f * Fy, jz = momentum<2>(P) + 0.5f * Fz;
    const Neq n = noneq_moments(P, drho, jx, jy, jz, M);
    float S6[6];
    const float s1 = M.s[1], sn = M.s[9], ir = M.inv_rho0;
    strain_yu(n, s1, sn, ir, S6);
    acc[0] += static_cast<double>(S6[0]) * S6[0] + static_cast<double>(S6[1]) * S6[1] +
              static_cast<double>(S6[2]) * S6[2] +
              2.0 * (static_cast<double>(S6[3]) * S6[3] + static_cast<double>(S6[4]) * S6[4] +
                     static_cast<double>(S6[5]) * S6[5]);
    // sigma = Y^T (2 W S): derivatives of Eq. LuoS with respect to m1, m9, m11, m13..15
    const float d0 = 2.0f * S6[0], d1 = 2.0f * S6[1], d2 = 2.0f * S6[2];
    const float d3 = 4.0f * S6[3], d4 = 4.0f * S6[4], d5 = 4.0f * S6[5];
    float sg[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) sg[k] = 0.0f;
    sg[1] = -s1 * ir * (1.0f / 38.0f) * (d0 + d1 + d2);
    sg[9] = sn * ir * (-0.5f * d0 + 0.25f * (d1 + d2));
    sg[11] = sn * ir * 0.75f * (d2 - d1);
    sg[13] = -1.5f * sn * ir * d3;
    sg[14] = -1.5f * sn * ir * d4;
    sg[15] = -1.5f * sn * ir * d5;
    // lam = T^T sigma - (dm^eq/dg)^T sigma,  (dm^eq/dg)^T sigma = a 1 + C^T b
    float lam[Q];
    apply_transpose(sg, lam);
    const float a = -11.0f * sg[1];
    const float bx = (38.0f * jx * sg[1] + 4.0f * jx * sg[9] + jy * sg[13] + jz * sg[15]) * ir;
    const float by = (38.0f * jy * sg[1] - 2.0f * jy * sg[9] + 2.0f * jy * sg[11] + jx * sg[13] + jz * sg[14]) * ir;
    const float bz = (38.0f * jz * sg[1] - 2.0f * jz * sg[9] - 2.0f * jz * sg[11] + jy * sg[14] + jx * sg[15]) * ir;
    static_for<Q>([&](auto ii) {
      constexpr int i = ii;
      lam[i] -= a + static_cast<float>(CX[i]) * bx + static_cast<float>(CY[i]) * by + static_cast<float>(CZ[i]) * bz;
    });
    store_local<Q>(lam_out, G, self * 4u, lam);
    if (grad_force) {
      grad_force[self] -= 0.5f * bx;
      grad_force[G.N + self] -= 0.5f * by;
      grad_force[2 * static_cast<size_t>(G.N) + self] -= 0.5f * bz;
    }
  }
  block_reduce_store(acc, partials);
}

// grad_u0 = sum_i lam0_i d g^eq_i / d u at (drho, u0): rho0 w_i (3 c_i + 9 (c_i.u) c_i - 3 u).
__global__ __launch_bounds__(kMaxBlock) void init_adjoint_kernel(Geo G, ModelF M, const float* __restrict__ rho_u,
                                                           const float* __restrict__ lam0, float* __restrict__ grad_u0) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= G.nx || y >= G.ny) return;
  const unsigned self = (static_cast<unsigned>(z) * G.ny + y) * G.nx + x;
  const size_t N = G.N;
  const float ux = rho_u[N + self], uy = rho_u[2 * N + self], uz = rho_u[3 * N + self];
  float gx = 0.f, gy = 0.f, gz = 0.f, sl = 0.f;
  static_for<Q>([&](auto ii) {
    constexpr int i = ii;
    const float l = lam0[i * N + self] * (static_cast<float>(W36[i]) / 36.0f);
    const float cu = static_cast<float>(CX[i]) * ux + static_cast<float>(CY[i]) * uy + static_cast<float>(CZ[i]) * uz;
    const float k = l * (3.0f + 9.0f * cu);
    gx += static_cast<float>(CX[i]) * k;
    gy += static_cast<float>(CY[i]) * k;
    gz += static_cast<float>(CZ[i]) * k;
    sl += l;
  });
  grad_u0[self] = M.rho0 * (gx - 3.0f * ux * sl);
  grad_u0[N + self] = M.rho0 * (gy - 3.0f * uy * sl);
  grad_u0[2 * N + self] = M.rho0 * (gz - 3.0f * uz * sl);
}

hipError_t launch_adjoint_step(const Geo& G, const ModelF& M, const ForceF& Fo, const float* j_n, const float* lam_in,
                               float* lam_out, float* grad_force, hipStream_t st) {
  const Launch L = node_launch(G);
  hipLaunchKernelGGL(adjoint_kernel, L.grid, L.block, 0, st, G, M, Fo, j_n, lam_in, lam_out, grad_force);
  return hipGetLastError();
}

hipError_t launch_loss_seed(int storage, const Geo& G, const ModelF& M, const ForceF& Fo, const void* buf,
                            float* lam_out, float* grad_force, double* partials, double* out, hipStream_t st) {
  unsigned nb = (G.N + 255) / 256;
  if (nb > static_cast<unsigned>(kReduceBlocks)) nb = kReduceBlocks;
  switch (storage) {
    case 0: hipLaunchKernelGGL(loss_seed_kernel<float>, dim3(nb), dim3(256), 0, st, G, M, Fo, static_cast<const float*>(buf), lam_out, grad_force, partials); break;
    case 1: hipLaunchKernelGGL(loss_seed_kernel<_Float16>, dim3(nb), dim3(256), 0, st, G, M, Fo, static_cast<const _Float16*>(buf), lam_out, grad_force, partials); break;
    case 2: hipLaunchKernelGGL(loss_seed_kernel<__bf16>, dim3(nb), dim3(256), 0, st, G, M, Fo, static_cast<const __bf16*>(buf), lam_out, grad_force, partials); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_final(partials, static_cast<int>(nb), out, st);
}

hipError_t launch_init_adjoint(const Geo& G, const ModelF& M, const float* rho_u, const float* lam0, float* grad_u0,
                               hipStream_t st) {
  const Launch L = node_launch(G);
  hipLaunchKernelGGL(init_adjoint_kernel, L.grid, L.block, 0, st, G, M, rho_u, lam0, grad_u0);
  return hipGetLastError();
}

}  // namespace d3q19
}  // namespace lbm
