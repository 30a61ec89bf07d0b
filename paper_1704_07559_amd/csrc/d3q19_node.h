// D3Q19 device helpers shared by the step kernel and the read-only kernels (strain query,
// diagnostics): the pull lattice, the body force at a node, the rates with a given s_nu,
// S:S, the force-corrected strain inputs and the implicit Smagorinsky rate.
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

// The force-corrected strain (optional) takes the non-equilibrium part plus half the Guo
// source, m - m^eq + S_F/2 (first-order Chapman-Enskog balance of the forced collision).
// StrainIn carries what the strain formulas read: ns, the moments for the Yu formula, and
// with CORR h = S_F/2, which the Chai formula adds as its own term: the Chai contraction of
// F-bar/2 is, in moment space, the Yu contraction of S_F/2 with the same rates (the identity
// of Section 5.1 holds for any vector). Without CORR, ns is the plain m - m^eq and nothing
// else is held, so the uncorrected step keeps its register budget.
template <bool CORR>
struct StrainIn {
  Neq ns;
  Neq h;
};

// SF: the Guo source T F-bar (read only with CORR).
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

// The read-only kernels (strain query, diagnostics) take the corrected form always, with a
// zero source when the correction is off (the same values as the plain form).
__device__ __forceinline__ StrainIn<true> strain_in_state(const Neq& n, float jx, float jy, float jz, float Fx,
                                                          float Fy, float Fz, const ModelF& M, const ForceF& Fo) {
  float SF[Q];
  if (Fo.strain_corr) {
    force_moments(jx, jy, jz, Fx, Fy, Fz, M.inv_rho0, SF);
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) SF[k] = 0.0f;
  }
  return strain_in<true>(n, SF);
}

// Chai strain (Eq. ChaiS) of the state with the given rates, force-corrected with CORR.
template <bool CORR>
__device__ __forceinline__ void strain_chai_in(const Pairs& P, float drho, float jx, float jy, float jz,
                                               const float (&rates)[Q], const StrainIn<CORR>& si, float inv_rho0,
                                               float (&S)[6]) {
  strain_chai(P, drho, jx, jy, jz, rates, inv_rho0, S);
  if constexpr (CORR) {
    float Sh[6];
    strain_yu(si.h, rates[1], rates[9], inv_rho0, Sh);
#pragma unroll
    for (int c = 0; c < 6; ++c) S[c] += Sh[c];
  }
}

// s_nu of the implicit Smagorinsky coupling at one node, from the formula V selects.
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

}  // namespace d3q19
}  // namespace lbm
