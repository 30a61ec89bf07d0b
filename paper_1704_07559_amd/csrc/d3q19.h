// D3Q19 He-Luo MRT model (Section 2 of the paper) and its two strain-rate formulas
// (Section 3), as per-node device functions.
//
// Tables: the velocity set of Eq. HeLuoD3Q19, the weights of Eq. omega and the
// transformation matrix T of Section 2, transcribed for this library. Everything else
// (row norms D_k = sum_i T_ki^2, opposite directions, the Chai contraction) is derived from
// them at compile time.
//
// Parity structure. For every opposite pair (a, b), c_b = -c_a, each row of T is either
// even (T_ka = T_kb: rows 0,1,2,9..15) or odd (T_ka = -T_kb: rows 3..8,16..18). The
// transforms therefore work on the pair sums s_p = g_a + g_b and differences
// d_p = g_a - g_b, which halves the arithmetic of both m = T g and g = T^-1 m
// (T^-1 = T^T D^-1 since the rows are orthogonal).
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"
#include "static_for.h"

namespace lbm {
namespace d3q19 {

constexpr int Q = 19;
constexpr int NP = 9;  // opposite pairs

constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};

// Weight numerators over 36: 1/3, 1/18 (i = 1..6), 1/36 (i = 7..18).
constexpr int W36[Q] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};

// Rows: delta_rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww,
//       p_xy, p_yz, p_xz, t_x, t_y, t_z.
constexpr int TM[Q][Q] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-30, -11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8},
    {12, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, -4, 4, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, -4, -4, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, -2, -2, 2, 2, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1},
};

// Strain components (xx, yy, zz, xy, yz, xz) as pairs of axes.
constexpr int SA[6] = {0, 1, 2, 0, 1, 0};
constexpr int SB[6] = {0, 1, 2, 1, 2, 2};

constexpr int cax(int axis, int i) { return axis == 0 ? CX[i] : (axis == 1 ? CY[i] : CZ[i]); }

struct Derived {
  int D[Q];        // row norms sum_i T_ki^2
  int opp[Q];      // opposite direction
  int pa[NP];      // first member of each pair (the lower index)
  int pb[NP];      // its opposite
  bool even[Q];    // row parity under i <-> opp(i)
  // Chai contraction: P[k][c] = sum_l c_la c_lb T_kl / D_k. N_c = sum_k s_k P[k][c] (T f)_k.
  double P[Q][6];
  bool ok;         // all rows orthogonal and of definite parity
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
      if (TM[k][r.pa[p]] != TM[k][r.pb[p]]) ev = false;
      if (TM[k][r.pa[p]] != -TM[k][r.pb[p]]) od = false;
    }
    if (!ev && !od) r.ok = false;
    if (od && TM[k][0] != 0) r.ok = false;
    r.even[k] = ev;
    for (int c = 0; c < 6; ++c) {
      int acc = 0;
      for (int l = 0; l < Q; ++l) acc += cax(SA[c], l) * cax(SB[c], l) * TM[k][l];
      r.P[k][c] = static_cast<double>(acc) / r.D[k];
    }
  }
  return r;
}

constexpr Derived DV = derive();
static_assert(DV.ok, "T must have orthogonal rows of definite parity");
static_assert(DV.D[0] == 19 && DV.D[1] == 2394 && DV.D[2] == 252 && DV.D[9] == 36 && DV.D[10] == 72,
              "row norms of T");
constexpr bool row_norms_match() {
  for (int k = 0; k < Q; ++k)
    if (DV.D[k] != kD3Q19RowNorm[k]) return false;
  return true;
}
static_assert(row_norms_match(), "the host's row norms (relaxation constants) must be those of T");

// ---------------------------------------------------------------------------------------
// Per-node state in registers
// ---------------------------------------------------------------------------------------

struct Pairs {
  float g0;
  float s[NP];  // g_a + g_b
  float d[NP];  // g_a - g_b
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

// A 1.0 the compiler cannot fold (an empty asm claims to change it; it lives in a scalar
// register). Written as fma(h, one, x), the sum of a population loaded from FP16 storage and
// an FP32 value becomes one mixed-precision FMA that reads the FP16 operand directly
// (v_fma_mix_f32), where h + x would first convert h (a plain add is not fused with the
// conversion). The result is the same rounded sum.
__device__ __forceinline__ float opaque_one() {
  float one = 1.0f;
  asm("" : "+s"(one));
  return one;
}

// Populations loaded from FP16 storage, kept two per register (pair order DV.pa / DV.pb) from
// the pull to the final sums: 10 registers instead of 19 live across the node update, which
// lets the FP16 step run 6 waves per SIMD instead of 5. The empty asm makes each packed pair
// opaque at the two places it is read, so that it is neither unpacked nor converted early
// (a conversion shared by the first and the last use would keep 19 FP32 values live again).
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
struct HalfPairs {
  h16x2 v[NP];
  _Float16 h0;
};

// g: the pulled populations, each converted from FP16 (so the narrowing here is exact).
__device__ __forceinline__ HalfPairs pack_pairs(const float (&g)[Q]) {
  HalfPairs hp;
  hp.h0 = static_cast<_Float16>(g[0]);
  asm("" : "+v"(hp.h0));
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    hp.v[p] = (h16x2){static_cast<_Float16>(g[DV.pa[p]]), static_cast<_Float16>(g[DV.pb[p]])};
    asm("" : "+v"(hp.v[p]));
  });
  return hp;
}

// make_pairs from the packed values: each sum and difference one mixed-precision FMA that
// reads its two FP16 operands from the halves of one register.
__device__ __forceinline__ Pairs make_pairs_packed(const HalfPairs& hp) {
  const float one = opaque_one();
  Pairs P;
  P.g0 = static_cast<float>(hp.h0);
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    const float a = static_cast<float>(hp.v[p].x), b = static_cast<float>(hp.v[p].y);
    P.s[p] = __builtin_fmaf(a, one, b);
    P.d[p] = __builtin_fmaf(b, -one, a);
  });
  return P;
}

// ---------------------------------------------------------------------------------------
// Factored transforms. The rows of T share partial sums of the pair sums and differences:
// the density, e and eps rows see only g_0, the sum over the six axis directions and the
// sum over the twelve diagonal ones; the stress rows see the axis pair sums and the sums of
// the diagonal pairs per coordinate plane; the momentum, heat-flux and ghost rows see the
// differences of the diagonal pairs per plane. Sharing them takes the forward transform
// from 111 to 62 FP32 operations per node against row-by-row evaluation over the pairs (the
// back-transform gains less: the compiler already shares most of its terms). Written once
// for any arithmetic type, so that the compile-time check below runs them on unit vectors
// against T itself.
// Pair order (DV.pa): (1,2) (3,4) (5,6) (7,10) (8,9) (11,14) (12,13) (15,18) (16,17).
// ---------------------------------------------------------------------------------------
template <typename F>
__host__ __device__ constexpr void forward_transform(F g0, const F (&s)[NP], const F (&d)[NP], F (&m)[Q]) {
  // even rows, from the pair sums
  const F A = s[3] + s[4];  // diagonals in the xy plane
  const F B = s[5] + s[6];  // xz plane
  const F C = s[7] + s[8];  // yz plane
  const F AB = A + B;
  const F Sdg = AB + C;  // all twelve diagonals
  const F s12 = s[1] + s[2];
  const F Sax = s[0] + s12;  // all six axis directions
  m[0] = (g0 + Sax) + Sdg;
  m[1] = F(-30) * g0 + (F(-11) * Sax + F(8) * Sdg);
  m[2] = F(12) * g0 + (F(-4) * Sax + Sdg);
  const F T1 = F(-2) * C + AB;
  m[9] = (F(2) * s[0] + T1) - s12;
  m[10] = F(-4) * s[0] + (F(2) * s12 + T1);
  const F D12 = s[1] - s[2];
  const F AmB = A - B;
  m[11] = D12 + AmB;
  m[12] = F(-2) * D12 + AmB;
  m[13] = s[3] - s[4];
  m[14] = s[7] - s[8];
  m[15] = s[5] - s[6];
  // odd rows, from the pair differences
  const F X1 = d[3] - d[4], X2 = d[5] - d[6];
  const F Y1 = d[3] + d[4], Y2 = d[7] - d[8];
  const F Z1 = d[5] + d[6], Z2 = d[7] + d[8];
  const F Xs = X1 + X2, Ys = Y1 + Y2, Zs = Z1 + Z2;
  m[3] = d[0] + Xs;
  m[4] = F(-4) * d[0] + Xs;
  m[5] = d[1] + Ys;
  m[6] = F(-4) * d[1] + Ys;
  m[7] = d[2] + Zs;
  m[8] = F(-4) * d[2] + Zs;
  m[16] = X1 - X2;
  m[17] = Y2 - Y1;
  m[18] = Z1 - Z2;
}

// dg = T^T w for rows 1..18 (row 0, the conserved density, is not read), as the change of
// g_0 and, for each pair (a, b), its even part e and odd part o: dg_a = e + o, dg_b = e - o.
template <typename F>
__host__ __device__ constexpr void back_transform(const F (&w)[Q], F& dg0, F (&e)[NP], F (&o)[NP]) {
  // even rows
  dg0 = F(-30) * w[1] + F(12) * w[2];
  const F Eax = F(-11) * w[1] + F(-4) * w[2];
  const F Edg = F(8) * w[1] + w[2];
  const F U = F(2) * w[10] - w[9];
  const F V = F(-2) * w[12] + w[11];
  const F EU = Eax + U;
  e[0] = F(-2) * U + Eax;
  e[1] = EU + V;
  e[2] = EU - V;
  const F W9 = w[9] + w[10], W11 = w[11] + w[12];
  const F EW = Edg + W9;
  const F Exy = EW + W11, Exz = EW - W11, Eyz = F(-2) * W9 + Edg;
  e[3] = Exy + w[13];
  e[4] = Exy - w[13];
  e[5] = Exz + w[15];
  e[6] = Exz - w[15];
  e[7] = Eyz + w[14];
  e[8] = Eyz - w[14];
  // odd rows
  o[0] = F(-4) * w[4] + w[3];
  o[1] = F(-4) * w[6] + w[5];
  o[2] = F(-4) * w[8] + w[7];
  const F Jx = w[3] + w[4], Jy = w[5] + w[6], Jz = w[7] + w[8];
  o[3] = (Jx + Jy) + (w[16] - w[17]);
  o[4] = (Jy - Jx) - (w[16] + w[17]);
  o[5] = (Jx + Jz) + (w[18] - w[16]);
  o[6] = (Jz - Jx) + (w[16] + w[18]);
  o[7] = (Jy + Jz) + (w[17] - w[18]);
  o[8] = (Jz - Jy) - (w[17] + w[18]);
}

// Both factored transforms reproduce T exactly on every unit vector.
constexpr bool transforms_match_T() {
  for (int i = 0; i < Q; ++i) {
    long long g0 = i == 0, s[NP] = {}, d[NP] = {}, m[Q] = {};
    for (int p = 0; p < NP; ++p) {
      const long long ga = DV.pa[p] == i, gb = DV.pb[p] == i;
      s[p] = ga + gb;
      d[p] = ga - gb;
    }
    forward_transform<long long>(g0, s, d, m);
    for (int k = 0; k < Q; ++k)
      if (m[k] != TM[k][i]) return false;
  }
  for (int k = 1; k < Q; ++k) {
    long long w[Q] = {}, dg0 = 0, e[NP] = {}, o[NP] = {};
    w[k] = 1;
    back_transform<long long>(w, dg0, e, o);
    if (dg0 != TM[k][0]) return false;
    for (int p = 0; p < NP; ++p)
      if (e[p] + o[p] != TM[k][DV.pa[p]] || e[p] - o[p] != TM[k][DV.pb[p]]) return false;
  }
  return true;
}
static_assert(transforms_match_T(), "factored transforms must equal T and T^T");

__device__ __forceinline__ void raw_moments(const Pairs& P, float (&m)[Q]) { forward_transform<float>(P.g0, P.s, P.d, m); }

// m_k = sum_i T_ki g_i. Every caller evaluates the same factored expressions, so the
// compiler shares them between the rows a kernel asks for.
template <int K>
__device__ __forceinline__ float moment(const Pairs& P) {
  float m[Q];
  raw_moments(P, m);
  return m[K];
}

// j_a = sum_i c_ia g_i (rows 3, 5, 7).
template <int AX>
__device__ __forceinline__ float momentum(const Pairs& P) {
  return moment<3 + 2 * AX>(P);
}

__device__ __forceinline__ float delta_rho(const Pairs& P) { return moment<0>(P); }

// Non-equilibrium moments m_k - m_k^eq for the non-conserved rows (Eq. meq, with rows 9..12
// as in the equilibrium column of Eq. solvem). Index k of the returned array is row k;
// rows 0, 3, 5, 7 are not filled.
// Rows relaxed with s_nu (Eq. sD3Q15meaning).
constexpr bool is_nu_slot(int k) { return k == 9 || k == 11 || k == 13 || k == 14 || k == 15; }

struct Neq {
  float m[Q];
};

__device__ __forceinline__ Neq noneq_moments(const Pairs& P, float drho, float jx, float jy, float jz,
                                             const ModelF& M) {
  Neq n;
  const float ir = M.inv_rho0;
  const float jx2 = jx * jx, jy2 = jy * jy, jz2 = jz * jz;
  const float jj = jx2 + jy2 + jz2;
  const float pxx = (2.0f * jx2 - jy2 - jz2) * ir;
  const float pww = (jy2 - jz2) * ir;
  n.m[1] = moment<1>(P) - (-11.0f * drho + 19.0f * jj * ir);
  n.m[2] = moment<2>(P) - (M.om_eps * drho + M.om_epsj * jj * ir);
  n.m[4] = moment<4>(P) + (2.0f / 3.0f) * jx;
  n.m[6] = moment<6>(P) + (2.0f / 3.0f) * jy;
  n.m[8] = moment<8>(P) + (2.0f / 3.0f) * jz;
  n.m[9] = moment<9>(P) - pxx;
  n.m[10] = moment<10>(P) - M.om_xx * pxx;
  n.m[11] = moment<11>(P) - pww;
  n.m[12] = moment<12>(P) - M.om_xx * pww;
  n.m[13] = moment<13>(P) - jx * jy * ir;
  n.m[14] = moment<14>(P) - jy * jz * ir;
  n.m[15] = moment<15>(P) - jx * jz * ir;
  n.m[16] = moment<16>(P);
  n.m[17] = moment<17>(P);
  n.m[18] = moment<18>(P);
  return n;
}

// Yu formula, Eq. LuoS (delta_t = 1, eps m^(1) = m - m^eq).
__device__ __forceinline__ void strain_yu(const Neq& n, float s1, float snu, float inv_rho0, float (&S)[6]) {
  const float a = s1 * n.m[1];
  const float b = snu * n.m[9];
  const float c = snu * n.m[11];
  S[0] = -(a + 19.0f * b) * (inv_rho0 * (1.0f / 38.0f));
  S[1] = -(2.0f * a - 19.0f * (b - 3.0f * c)) * (inv_rho0 * (1.0f / 76.0f));
  S[2] = -(2.0f * a - 19.0f * (b + 3.0f * c)) * (inv_rho0 * (1.0f / 76.0f));
  S[3] = -1.5f * snu * n.m[13] * inv_rho0;
  S[4] = -1.5f * snu * n.m[14] * inv_rho0;
  S[5] = -1.5f * snu * n.m[15] * inv_rho0;
}

// Chai formula, Eq. ChaiS: S = -sum_i c_i c_i (T^-1 Lambda-hat T)_ij f_j^neq / (2 rho0 c_s^2).
// f^neq = g - g^eq(delta_rho, j) is formed in distribution space (the delta-rho form of
// Eq. edf); the contraction (c c)^T T^-1 Lambda-hat T is precomputed per rate group. Only
// even rows contribute (c c is even under i <-> opp(i)), so the contraction acts on the
// pair sums of f^neq. `rates` are the Lambda-hat entries of rows 0..18 at this node.
__device__ __forceinline__ void strain_chai(const Pairs& P, float drho, float jx, float jy, float jz,
                                            const float (&rates)[Q], float inv_rho0, float (&S)[6]) {
  const float jj = (jx * jx + jy * jy + jz * jz) * inv_rho0;
  // g^eq_0 and g^eq_a + g^eq_b for each pair (the odd c.u term cancels in the sum).
  const float base = drho - 1.5f * jj;
  float fn0 = P.g0 - (12.0f / 36.0f) * base;
  float fs[NP];
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    constexpr int a = DV.pa[p];
    const float cj = static_cast<float>(CX[a]) * jx + static_cast<float>(CY[a]) * jy + static_cast<float>(CZ[a]) * jz;
    const float geq_sum = (2.0f * W36[a] / 36.0f) * (base + 4.5f * cj * cj * inv_rho0);
    fs[p] = P.s[p] - geq_sum;
  });
  // (T f^neq)_k for the even rows with a non-zero second-moment projection.
  float N[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    if constexpr (DV.even[k] && (DV.P[k][0] != 0.0 || DV.P[k][1] != 0.0 || DV.P[k][2] != 0.0 ||
                                 DV.P[k][3] != 0.0 || DV.P[k][4] != 0.0 || DV.P[k][5] != 0.0)) {
      float tf = -0.0f;
      tf = acc_int<TM[k][0]>(tf, fn0);
      static_for<NP>([&](auto pi) {
        constexpr int p = pi;
        tf = acc_int<TM[k][DV.pa[p]]>(tf, fs[p]);
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

// The implicit Smagorinsky rate at one node from the Yu strain of the non-equilibrium
// moments (the Chai strain is the same function of the state, Section 5.1).
__device__ __forceinline__ float implicit_rate_yu(const Neq& n, const ModelF& M, const ViscF& V) {
  float P[6], A[6];
  strain_yu(n, M.s[1], 0.0f, M.inv_rho0, P);
  strain_yu(n, 0.0f, 1.0f, M.inv_rho0, A);
  return implicit_smagorinsky(P, A, V.nu0, V.csmag2);
}

// Guo force moments S_F = T F-bar with F-bar_i = (d g^eq_i / d j) . F (He-Luo equilibrium
// with the paper's omega values in T g^eq), rows 0..18.
__device__ __forceinline__ void force_moments(float jx, float jy, float jz, float Fx, float Fy, float Fz,
                                              float inv_rho0, float (&SF)[Q]) {
  const float jF = (jx * Fx + jy * Fy + jz * Fz) * inv_rho0;
  const float p9 = (4.0f * jx * Fx - 2.0f * jy * Fy - 2.0f * jz * Fz) * inv_rho0;
  const float p11 = (2.0f * jy * Fy - 2.0f * jz * Fz) * inv_rho0;
  SF[0] = 0.f;
  SF[1] = 38.0f * jF;
  SF[2] = -11.0f * jF;
  SF[3] = Fx;
  SF[4] = (-2.0f / 3.0f) * Fx;
  SF[5] = Fy;
  SF[6] = (-2.0f / 3.0f) * Fy;
  SF[7] = Fz;
  SF[8] = (-2.0f / 3.0f) * Fz;
  SF[9] = p9;
  SF[10] = -0.5f * p9;
  SF[11] = p11;
  SF[12] = -0.5f * p11;
  SF[13] = (jx * Fy + jy * Fx) * inv_rho0;
  SF[14] = (jy * Fz + jz * Fy) * inv_rho0;
  SF[15] = (jx * Fz + jz * Fx) * inv_rho0;
  SF[16] = 0.f;
  SF[17] = 0.f;
  SF[18] = 0.f;
}

// g += T^T w for rows 1..18 (w[0] is not read: the density row is conserved by every
// collision and every initial non-equilibrium part).
__device__ __forceinline__ void add_scaled_back_transform(const float (&w)[Q], float (&g)[Q]) {
  float dg0, e[NP], o[NP];
  back_transform<float>(w, dg0, e, o);
  g[0] += dg0;
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    g[DV.pa[p]] += e[p] + o[p];
    g[DV.pb[p]] += e[p] - o[p];
  });
}

// The same sums from the packed FP16 pre-collision populations, g = hp + T^T w, as
// mixed-precision FMAs (the same rounded sums as above).
__device__ __forceinline__ void add_scaled_back_transform_packed(const float (&w)[Q], const HalfPairs& hp,
                                                                 float (&g)[Q]) {
  float dg0, e[NP], o[NP];
  back_transform<float>(w, dg0, e, o);
  const float one = opaque_one();
  _Float16 h0 = hp.h0;
  asm("" : "+v"(h0));
  g[0] = __builtin_fmaf(static_cast<float>(h0), one, dg0);
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    h16x2 v = hp.v[p];
    asm("" : "+v"(v));
    g[DV.pa[p]] = __builtin_fmaf(static_cast<float>(v.x), one, e[p] + o[p]);
    g[DV.pb[p]] = __builtin_fmaf(static_cast<float>(v.y), one, e[p] - o[p]);
  });
}

// g += T^-1 dm = T^T (D^-1 dm) for rows 1..18 (dm[0] is not read).
__device__ __forceinline__ void add_back_transform(const float (&dm)[Q], float (&g)[Q]) {
  float w[Q];
  w[0] = 0.0f;
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    if constexpr (k > 0) w[k] = dm[k] * (1.0f / static_cast<float>(DV.D[k]));
  });
  add_scaled_back_transform(w, g);
}

// Canonical populations from a non-equilibrium moment vector (rows given, others zero):
// g_i += sum_k T_ki mn_k / D_k. Used for the Chapman-Enskog initial state.
__device__ __forceinline__ void add_neq_from_moments(const float (&mn)[Q], float (&g)[Q]) { add_back_transform(mn, g); }

// g^eq_i(delta_rho, j), the delta-rho form of Eq. edf with u = j / rho0.
__device__ __forceinline__ void equilibrium(float drho, float jx, float jy, float jz, float inv_rho0, float (&g)[Q]) {
  const float jj = (jx * jx + jy * jy + jz * jz) * inv_rho0;
  const float base = drho - 1.5f * jj;
  static_for<Q>([&](auto ii) {
    constexpr int i = ii;
    const float cj = static_cast<float>(CX[i]) * jx + static_cast<float>(CY[i]) * jy + static_cast<float>(CZ[i]) * jz;
    g[i] = (static_cast<float>(W36[i]) / 36.0f) * (base + 3.0f * cj + 4.5f * cj * cj * inv_rho0);
  });
}

}  // namespace d3q19
}  // namespace lbm
