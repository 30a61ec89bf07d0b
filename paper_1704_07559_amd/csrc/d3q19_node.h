// D3Q19 device helpers shared by the step kernel and the read-only kernels (strain query,
// diagnostics): the pull lattice, the body force at a node, the rates with a given s_nu,
// S:S, and the implicit Smagorinsky rate.
#pragma once
#include <hip/hip_runtime.h>

#include "d3q19.h"
#include "internal.h"

namespace lbm {
namespace d3q19 {

struct Lat {
  static constexpr int Q = 19;
  static constexpr int cx(int i) { return CX[i]; }
  static constexpr int cy(int i) { return CY[i]; }
  static constexpr int cz(int i) { return CZ[i]; }
  static constexpr int opp(int i) { return DV.opp[i]; }
};

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

// s_nu of the implicit Smagorinsky coupling at one node, from the formula V selects.
__device__ __forceinline__ float implicit_rate(const Pairs& P_, float drho, float jx, float jy, float jz, const Neq& n,
                                               const ModelF& M, const ViscF& V) {
  float P[6], A[6];
  if (V.drive_chai) {
    float rb[Q], rn[Q];
    rates_with(M, 0.0f, rb);
    static_for<Q>([&](auto ki) {
      constexpr int k = ki;
      rn[k] = is_nu_slot(k) ? 1.0f : 0.0f;
    });
    strain_chai(P_, drho, jx, jy, jz, rb, M.inv_rho0, P);
    strain_chai(P_, drho, jx, jy, jz, rn, M.inv_rho0, A);
  } else {
    strain_yu(n, M.s[1], 0.0f, M.inv_rho0, P);
    strain_yu(n, 0.0f, 1.0f, M.inv_rho0, A);
  }
  return implicit_smagorinsky(P, A, V.nu0, V.csmag2);
}

}  // namespace d3q19
}  // namespace lbm
