// D2Q9 MRT model with the paper's delta-rho He-Luo equilibrium, the Chai formula
// (Eq. ChaiS, which Section 5.3 says holds on D2Q9) and the Yu-type formula obtained by
// the route of Section 5.4. The velocity set, weights and transformation matrix are the
// Lallemand-Luo choice (outside the paper): velocities 0, E, N, W, S, NE, NW, SW, SE;
// moment rows rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy. Strain order: xx, yy, xy.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"
#include "static_for.h"

namespace lbm {
namespace d2q9 {

constexpr int Q = 9;
constexpr int NP = 4;

constexpr int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int W36[Q] = {16, 4, 4, 4, 4, 1, 1, 1, 1};  // 4/9, 1/9, 1/36

constexpr int TM[Q][Q] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

constexpr int SA[3] = {0, 1, 0};
constexpr int SB[3] = {0, 1, 1};
constexpr int cax(int axis, int i) { return axis == 0 ? CX[i] : CY[i]; }

struct Derived {
  int D[Q];
  int opp[Q];
  int pa[NP], pb[NP];
  bool even[Q];
  double P[Q][3];  // sum_l c_la c_lb T_kl / D_k
  bool ok;
};

constexpr Derived derive() {
  Derived r{};
  r.ok = true;
  for (int k = 0; k < Q; ++k) {
    int s = 0;
    for (int i = 0; i < Q; ++i) s += TM[k][i] * TM[k][i];
    r.D[k] = s;
    for (int k2 = 0; k2 < Q; ++k2) {
      if (k2 == k) continue;
      int dot = 0;
      for (int i = 0; i < Q; ++i) dot += TM[k][i] * TM[k2][i];
      if (dot != 0) r.ok = false;
    }
  }
  for (int i = 0; i < Q; ++i) {
    r.opp[i] = -1;
    for (int j = 0; j < Q; ++j)
      if (CX[j] == -CX[i] && CY[j] == -CY[i]) r.opp[i] = j;
    if (r.opp[i] < 0) r.ok = false;
  }
  int np = 0;
  for (int i = 1; i < Q; ++i)
    if (i < r.opp[i]) {
      r.pa[np] = i;
      r.pb[np] = r.opp[i];
      ++np;
    }
  if (np != NP) r.ok = false;
  for (int k = 0; k < Q; ++k) {
    bool ev = true, od = true;
    for (int p = 0; p < NP; ++p) {
      if (TM[k][r.pa[p]] != TM[k][r.pb[p]]) ev = false;
      if (TM[k][r.pa[p]] != -TM[k][r.pb[p]]) od = false;
    }
    if (!ev && !od) r.ok = false;
    if (od && TM[k][0] != 0) r.ok = false;
    r.even[k] = ev;
    for (int c = 0; c < 3; ++c) {
      int acc = 0;
      for (int l = 0; l < Q; ++l) acc += cax(SA[c], l) * cax(SB[c], l) * TM[k][l];
      r.P[k][c] = static_cast<double>(acc) / r.D[k];
    }
  }
  return r;
}

constexpr Derived DV = derive();
static_assert(DV.ok, "D2Q9 T must have orthogonal rows of definite parity");
static_assert(DV.D[0] == 9 && DV.D[1] == 36 && DV.D[2] == 36 && DV.D[7] == 4 && DV.D[8] == 4, "row norms of T");

struct Lat {
  static constexpr int Q = 9;
  static constexpr int cx(int i) { return CX[i]; }
  static constexpr int cy(int i) { return CY[i]; }
  static constexpr int cz(int) { return 0; }
  static constexpr int opp(int i) { return DV.opp[i]; }
};

constexpr bool is_nu_slot(int k) { return k == 7 || k == 8; }

struct Pairs {
  float g0;
  float s[NP];
  float d[NP];
};

__device__ __forceinline__ Pairs make_pairs(const float (&g)[Q]) {
  Pairs P;
  P.g0 = g[0];
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    P.s[p] = g[DV.pa[p]] + g[DV.pb[p]];
    P.d[p] = g[DV.pa[p]] - g[DV.pb[p]];
  });
  return P;
}

template <int K>
__device__ __forceinline__ float moment(const Pairs& P) {
  float acc = -0.0f;
  if constexpr (DV.even[K]) {
    acc = acc_int<TM[K][0]>(acc, P.g0);
    static_for<NP>([&](auto pi) {
      constexpr int p = pi;
      acc = acc_int<TM[K][DV.pa[p]]>(acc, P.s[p]);
    });
  } else {
    static_for<NP>([&](auto pi) {
      constexpr int p = pi;
      acc = acc_int<TM[K][DV.pa[p]]>(acc, P.d[p]);
    });
  }
  return acc;
}

template <int AX>
__device__ __forceinline__ float momentum(const Pairs& P) {
  float acc = -0.0f;
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    acc = acc_int<cax(AX, DV.pa[p])>(acc, P.d[p]);
  });
  return acc;
}

__device__ __forceinline__ float delta_rho(const Pairs& P) {
  float acc = P.g0;
  static_for<NP>([&](auto pi) { acc += P.s[decltype(pi)::value]; });
  return acc;
}

struct Neq {
  float m[Q];
};

// m - m^eq for the non-conserved rows 1, 2, 4, 6, 7, 8 (m^eq = T g^eq of the He-Luo
// equilibrium: e = -2 drho + 3|j|^2/rho0, eps = drho - 3|j|^2/rho0, q = -j,
// p_xx = (j_x^2 - j_y^2)/rho0, p_xy = j_x j_y / rho0).
__device__ __forceinline__ Neq noneq_moments(const Pairs& P, float drho, float jx, float jy, float inv_rho0) {
  Neq n;
  const float jj = (jx * jx + jy * jy) * inv_rho0;
  n.m[1] = moment<1>(P) - (-2.0f * drho + 3.0f * jj);
  n.m[2] = moment<2>(P) - (drho - 3.0f * jj);
  n.m[4] = moment<4>(P) + jx;
  n.m[6] = moment<6>(P) + jy;
  n.m[7] = moment<7>(P) - (jx * jx - jy * jy) * inv_rho0;
  n.m[8] = moment<8>(P) - jx * jy * inv_rho0;
  return n;
}

// Yu-type formula (Section 5.4 applied to this basis):
// S_xx,yy = -(s_e m1 +/- 3 s_nu m7) / (4 rho0), S_xy = -3 s_nu m8 / (2 rho0).
__device__ __forceinline__ void strain_yu(const Neq& n, float se, float snu, float inv_rho0, float (&S)[3]) {
  const float a = se * n.m[1], b = 3.0f * snu * n.m[7];
  S[0] = -(a + b) * 0.25f * inv_rho0;
  S[1] = -(a - b) * 0.25f * inv_rho0;
  S[2] = -1.5f * snu * n.m[8] * inv_rho0;
}

// Chai formula (Eq. ChaiS) from f^neq = g - g^eq, contraction on the pair sums.
__device__ __forceinline__ void strain_chai(const Pairs& P, float drho, float jx, float jy, const float (&rates)[Q],
                                            float inv_rho0, float (&S)[3]) {
  const float jj = (jx * jx + jy * jy) * inv_rho0;
  const float base = drho - 1.5f * jj;
  const float fn0 = P.g0 - (16.0f / 36.0f) * base;
  float fs[NP];
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    constexpr int a = DV.pa[p];
    const float cj = static_cast<float>(CX[a]) * jx + static_cast<float>(CY[a]) * jy;
    fs[p] = P.s[p] - (2.0f * W36[a] / 36.0f) * (base + 4.5f * cj * cj * inv_rho0);
  });
  float N[3] = {0.f, 0.f, 0.f};
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    if constexpr (DV.even[k] && (DV.P[k][0] != 0.0 || DV.P[k][1] != 0.0 || DV.P[k][2] != 0.0)) {
      float tf = -0.0f;
      tf = acc_int<TM[k][0]>(tf, fn0);
      static_for<NP>([&](auto pi) {
        constexpr int p = pi;
        tf = acc_int<TM[k][DV.pa[p]]>(tf, fs[p]);
      });
      const float w = rates[k] * tf;
      static_for<3>([&](auto ci) {
        constexpr int c = ci;
        if constexpr (DV.P[k][c] != 0.0) N[c] = __builtin_fmaf(static_cast<float>(DV.P[k][c]), w, N[c]);
      });
    }
  });
  static_for<3>([&](auto ci) {
    constexpr int c = ci;
    S[c] = -1.5f * inv_rho0 * N[c];
  });
}

__device__ __forceinline__ void force_moments(float jx, float jy, float Fx, float Fy, float inv_rho0, float (&SF)[Q]) {
  const float jF = (jx * Fx + jy * Fy) * inv_rho0;
  SF[0] = 0.f;
  SF[1] = 6.0f * jF;
  SF[2] = -6.0f * jF;
  SF[3] = Fx;
  SF[4] = -Fx;
  SF[5] = Fy;
  SF[6] = -Fy;
  SF[7] = 2.0f * (jx * Fx - jy * Fy) * inv_rho0;
  SF[8] = (jx * Fy + jy * Fx) * inv_rho0;
}

__device__ __forceinline__ void add_back_transform(const float (&dm)[Q], float (&g)[Q]) {
  float w[Q];
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    w[k] = dm[k] * (1.0f / static_cast<float>(DV.D[k]));
  });
  float r0 = -0.0f;
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    if constexpr (DV.even[k]) r0 = acc_int<TM[k][0]>(r0, w[k]);
  });
  g[0] += r0;
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    constexpr int a = DV.pa[p];
    constexpr int b = DV.pb[p];
    float e = -0.0f, o = -0.0f;
    static_for<Q>([&](auto ki) {
      constexpr int k = ki;
      if constexpr (DV.even[k]) e = acc_int<TM[k][a]>(e, w[k]);
      else o = acc_int<TM[k][a]>(o, w[k]);
    });
    g[a] += e + o;
    g[b] += e - o;
  });
}

__device__ __forceinline__ void equilibrium(float drho, float jx, float jy, float inv_rho0, float (&g)[Q]) {
  const float jj = (jx * jx + jy * jy) * inv_rho0;
  const float base = drho - 1.5f * jj;
  static_for<Q>([&](auto ii) {
    constexpr int i = ii;
    const float cj = static_cast<float>(CX[i]) * jx + static_cast<float>(CY[i]) * jy;
    g[i] = (static_cast<float>(W36[i]) / 36.0f) * (base + 3.0f * cj + 4.5f * cj * cj * inv_rho0);
  });
}

}  // namespace d2q9
}  // namespace lbm
