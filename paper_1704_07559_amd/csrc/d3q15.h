// D3Q15 MRT model with the paper's delta-rho equilibrium (Eq. edf with the D3Q15 weights),
// the Chai formula (Eq. ChaiS, which Section 5.3 says holds on D3Q15) and the Yu-type
// formula obtained by the route of Section 5.4. The paper gives no D3Q15 matrix; the basis
// is the d'Humieres et al. (2002) one (outside the paper), generated here at compile time
// from its definition as polynomials of the velocity:
//   rho 1 | e c^2 - 2 | eps (15 c^4 - 55 c^2 + 32)/2 | j_a c_a | q_a c_a (5 c^2 - 13)/2 |
//   3p_xx 2c_x^2 - c_y^2 - c_z^2 | p_ww c_y^2 - c_z^2 | p_ab c_a c_b | m_xyz c_x c_y c_z
// rows ordered rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, p_ww, p_xy, p_yz, p_xz,
// m_xyz. Velocities: rest, six faces, eight corners, opposite pairs adjacent. Weights
// 2/9, 1/9, 1/72. Strain order xx, yy, zz, xy, yz, xz.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"
#include "static_for.h"

namespace lbm {
namespace d3q15 {

constexpr int Q = 15;
constexpr int NP = 7;

constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};
constexpr int W72[Q] = {16, 8, 8, 8, 8, 8, 8, 1, 1, 1, 1, 1, 1, 1, 1};  // 2/9, 1/9, 1/72

struct Basis {
  int v[Q][Q];
};

constexpr Basis make_basis() {
  Basis b{};
  for (int i = 0; i < Q; ++i) {
    const int x = CX[i], y = CY[i], z = CZ[i];
    const int c2 = x * x + y * y + z * z;
    const int row[Q] = {1,
                        c2 - 2,
                        (15 * c2 * c2 - 55 * c2 + 32) / 2,
                        x,
                        x * (5 * c2 - 13) / 2,
                        y,
                        y * (5 * c2 - 13) / 2,
                        z,
                        z * (5 * c2 - 13) / 2,
                        2 * x * x - y * y - z * z,
                        y * y - z * z,
                        x * y,
                        y * z,
                        x * z,
                        x * y * z};
    for (int k = 0; k < Q; ++k) b.v[k][i] = row[k];
  }
  return b;
}

constexpr Basis TB = make_basis();

constexpr int SA[6] = {0, 1, 2, 0, 1, 0};
constexpr int SB[6] = {0, 1, 2, 1, 2, 2};
constexpr int cax(int axis, int i) { return axis == 0 ? CX[i] : (axis == 1 ? CY[i] : CZ[i]); }

struct Derived {
  int D[Q];
  int opp[Q];
  int pa[NP], pb[NP];
  bool even[Q];
  double P[Q][6];  // sum_l c_la c_lb T_kl / D_k
  bool ok;
};

constexpr Derived derive() {
  Derived r{};
  r.ok = true;
  for (int k = 0; k < Q; ++k) {
    int s = 0;
    for (int i = 0; i < Q; ++i) s += TB.v[k][i] * TB.v[k][i];
    r.D[k] = s;
    for (int k2 = 0; k2 < Q; ++k2) {
      if (k2 == k) continue;
      int dot = 0;
      for (int i = 0; i < Q; ++i) dot += TB.v[k][i] * TB.v[k2][i];
      if (dot != 0) r.ok = false;
    }
  }
  for (int i = 0; i < Q; ++i) {
    r.opp[i] = -1;
    for (int j = 0; j < Q; ++j)
      if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) r.opp[i] = j;
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
      if (TB.v[k][r.pa[p]] != TB.v[k][r.pb[p]]) ev = false;
      if (TB.v[k][r.pa[p]] != -TB.v[k][r.pb[p]]) od = false;
    }
    if (!ev && !od) r.ok = false;
    if (od && TB.v[k][0] != 0) r.ok = false;
    r.even[k] = ev;
    for (int c = 0; c < 6; ++c) {
      int acc = 0;
      for (int l = 0; l < Q; ++l) acc += cax(SA[c], l) * cax(SB[c], l) * TB.v[k][l];
      r.P[k][c] = static_cast<double>(acc) / r.D[k];
    }
  }
  return r;
}

constexpr Derived DV = derive();
static_assert(DV.ok, "D3Q15 T must have orthogonal rows of definite parity");
static_assert(DV.D[0] == 15 && DV.D[1] == 18 && DV.D[2] == 360 && DV.D[4] == 40 && DV.D[9] == 12 &&
                  DV.D[10] == 4 && DV.D[11] == 8 && DV.D[14] == 8,
              "row norms of the d'Humieres D3Q15 basis");

struct Lat {
  static constexpr int Q = 15;
  static constexpr int cx(int i) { return CX[i]; }
  static constexpr int cy(int i) { return CY[i]; }
  static constexpr int cz(int i) { return CZ[i]; }
  static constexpr int opp(int i) { return DV.opp[i]; }
};

constexpr bool is_nu_slot(int k) { return k >= 9 && k <= 13; }

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
    acc = acc_int<TB.v[K][0]>(acc, P.g0);
    static_for<NP>([&](auto pi) {
      constexpr int p = pi;
      acc = acc_int<TB.v[K][DV.pa[p]]>(acc, P.s[p]);
    });
  } else {
    static_for<NP>([&](auto pi) {
      constexpr int p = pi;
      acc = acc_int<TB.v[K][DV.pa[p]]>(acc, P.d[p]);
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

// m - m^eq for the non-conserved rows (m^eq = T g^eq: e = -drho + |j|^2/rho0,
// eps = drho - 5|j|^2/rho0, q = -7 j / 3, 3p_xx = (2j_x^2 - j_y^2 - j_z^2)/rho0,
// p_ww = (j_y^2 - j_z^2)/rho0, p_ab = j_a j_b / rho0, m_xyz = 0).
__device__ __forceinline__ Neq noneq_moments(const Pairs& P, float drho, float jx, float jy, float jz,
                                             float inv_rho0) {
  Neq n;
  const float jx2 = jx * jx, jy2 = jy * jy, jz2 = jz * jz;
  const float jj = (jx2 + jy2 + jz2) * inv_rho0;
  n.m[1] = moment<1>(P) - (jj - drho);
  n.m[2] = moment<2>(P) - (drho - 5.0f * jj);
  n.m[4] = __builtin_fmaf(7.0f / 3.0f, jx, moment<4>(P));
  n.m[6] = __builtin_fmaf(7.0f / 3.0f, jy, moment<6>(P));
  n.m[8] = __builtin_fmaf(7.0f / 3.0f, jz, moment<8>(P));
  n.m[9] = moment<9>(P) - (2.0f * jx2 - jy2 - jz2) * inv_rho0;
  n.m[10] = moment<10>(P) - (jy2 - jz2) * inv_rho0;
  n.m[11] = moment<11>(P) - jx * jy * inv_rho0;
  n.m[12] = moment<12>(P) - jy * jz * inv_rho0;
  n.m[13] = moment<13>(P) - jx * jz * inv_rho0;
  n.m[14] = moment<14>(P);
  return n;
}

// Yu-type formula (Section 5.4 on this basis):
// S_xx = -(s_e m1 + s_nu m9) / (2 rho0), S_yy,zz = -(2 s_e m1 - s_nu m9 +/- 3 s_nu m10) / (4 rho0),
// S_xy,yz,xz = -3 s_nu m11,12,13 / (2 rho0).
__device__ __forceinline__ void strain_yu(const Neq& n, float se, float snu, float inv_rho0, float (&S)[6]) {
  const float a = se * n.m[1], b = snu * n.m[9], c = 3.0f * snu * n.m[10];
  S[0] = -(a + b) * (0.5f * inv_rho0);
  S[1] = -(2.0f * a - b + c) * (0.25f * inv_rho0);
  S[2] = -(2.0f * a - b - c) * (0.25f * inv_rho0);
  S[3] = -1.5f * snu * n.m[11] * inv_rho0;
  S[4] = -1.5f * snu * n.m[12] * inv_rho0;
  S[5] = -1.5f * snu * n.m[13] * inv_rho0;
}

// Chai formula (Eq. ChaiS) from f^neq = g - g^eq in distribution space; only even rows
// contribute (c c is even under i <-> opp(i)), so the contraction acts on pair sums.
__device__ __forceinline__ void strain_chai(const Pairs& P, float drho, float jx, float jy, float jz,
                                            const float (&rates)[Q], float inv_rho0, float (&S)[6]) {
  const float jj = (jx * jx + jy * jy + jz * jz) * inv_rho0;
  const float base = drho - 1.5f * jj;
  const float fn0 = P.g0 - (static_cast<float>(W72[0]) / 72.0f) * base;
  float fs[NP];
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    constexpr int a = DV.pa[p];
    const float cj = static_cast<float>(CX[a]) * jx + static_cast<float>(CY[a]) * jy + static_cast<float>(CZ[a]) * jz;
    fs[p] = P.s[p] - (2.0f * W72[a] / 72.0f) * (base + 4.5f * cj * cj * inv_rho0);
  });
  float N[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    if constexpr (DV.even[k] && (DV.P[k][0] != 0.0 || DV.P[k][1] != 0.0 || DV.P[k][2] != 0.0 || DV.P[k][3] != 0.0 ||
                                 DV.P[k][4] != 0.0 || DV.P[k][5] != 0.0)) {
      float tf = -0.0f;
      tf = acc_int<TB.v[k][0]>(tf, fn0);
      static_for<NP>([&](auto pi) {
        constexpr int p = pi;
        tf = acc_int<TB.v[k][DV.pa[p]]>(tf, fs[p]);
      });
      const float w = rates[k] * tf;
      static_for<6>([&](auto ci) {
        constexpr int c = ci;
        if constexpr (DV.P[k][c] != 0.0) N[c] = __builtin_fmaf(static_cast<float>(DV.P[k][c]), w, N[c]);
      });
    }
  });
  static_for<6>([&](auto ci) {
    constexpr int c = ci;
    S[c] = -1.5f * inv_rho0 * N[c];
  });
}

// Guo force moments S_F = T F-bar, F-bar = (d g^eq / d j) . F.
__device__ __forceinline__ void force_moments(float jx, float jy, float jz, float Fx, float Fy, float Fz, float inv_rho0,
                                              float (&SF)[Q]) {
  const float jF = (jx * Fx + jy * Fy + jz * Fz) * inv_rho0;
  SF[0] = 0.f;
  SF[1] = 2.0f * jF;
  SF[2] = -10.0f * jF;
  SF[3] = Fx;
  SF[4] = (-7.0f / 3.0f) * Fx;
  SF[5] = Fy;
  SF[6] = (-7.0f / 3.0f) * Fy;
  SF[7] = Fz;
  SF[8] = (-7.0f / 3.0f) * Fz;
  SF[9] = (4.0f * jx * Fx - 2.0f * jy * Fy - 2.0f * jz * Fz) * inv_rho0;
  SF[10] = (2.0f * jy * Fy - 2.0f * jz * Fz) * inv_rho0;
  SF[11] = (jx * Fy + jy * Fx) * inv_rho0;
  SF[12] = (jy * Fz + jz * Fy) * inv_rho0;
  SF[13] = (jx * Fz + jz * Fx) * inv_rho0;
  SF[14] = 0.f;
}

// g += T^-1 dm = T^T (D^-1 dm), on pair sums and differences.
__device__ __forceinline__ void add_back_transform(const float (&dm)[Q], float (&g)[Q]) {
  float w[Q];
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    w[k] = dm[k] * (1.0f / static_cast<float>(DV.D[k]));
  });
  float r0 = -0.0f;
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    if constexpr (DV.even[k]) r0 = acc_int<TB.v[k][0]>(r0, w[k]);
  });
  g[0] += r0;
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    constexpr int a = DV.pa[p];
    constexpr int b = DV.pb[p];
    float e = -0.0f, o = -0.0f;
    static_for<Q>([&](auto ki) {
      constexpr int k = ki;
      if constexpr (DV.even[k]) e = acc_int<TB.v[k][a]>(e, w[k]);
      else o = acc_int<TB.v[k][a]>(o, w[k]);
    });
    g[a] += e + o;
    g[b] += e - o;
  });
}

__device__ __forceinline__ void equilibrium(float drho, float jx, float jy, float jz, float inv_rho0, float (&g)[Q]) {
  const float jj = (jx * jx + jy * jy + jz * jz) * inv_rho0;
  const float base = drho - 1.5f * jj;
  static_for<Q>([&](auto ii) {
    constexpr int i = ii;
    const float cj = static_cast<float>(CX[i]) * jx + static_cast<float>(CY[i]) * jy + static_cast<float>(CZ[i]) * jz;
    g[i] = (static_cast<float>(W72[i]) / 72.0f) * (base + 3.0f * cj + 4.5f * cj * cj * inv_rho0);
  });
}

}  // namespace d3q15
}  // namespace lbm
