// Discrete adjoint of the D3Q19 step and of the strain-squared loss, for a constant or a
// strain-dependent viscosity.
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
//
// Strain-dependent viscosity: L = L(s_new) with s_new a function of the strain of Eq. LuoS,
// S = (Y_e + s Y_n) m^neq (affine in the rate s it is taken with). Lagged kinds: s = the
// s_nu field (state), s_new = h(|S|), h = 1/(3 nu + 1/2), and s_new becomes the next field;
// implicit kind: s = s_new solves s (3 nu(|S(s)|) + 1/2) = 1. The step's transpose gains a
// rank-one term: sigma = dJ/ds_new = -sum_{k nu rows} mu_k (m^neq_k + S_F,k / 2) (+ the
// adjoint of the field s_new is written to), then dJ/dm^neq = Y(s)^T (c dgamma/dS) with
// c = sigma h'(gamma) (lagged) or -sigma s k / (dG/ds) (implicit, k = 3 C_s^2), mapped through
// m^neq = m - m^eq(drho, j).
#include <hip/hip_runtime.h>

#include "d3q19.h"
#include "internal.h"
#include "launch.h"
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
  // rows 1..18 by the factored back-transform, row 0 (all ones) added to every direction
  float dg0, e[NP], o[NP];
  back_transform<float>(v, dg0, e, o);
  out[0] = dg0 + v[0];
  static_for<NP>([&](auto pi) {
    constexpr int p = pi;
    const float ep = e[p] + v[0];
    out[DV.pa[p]] = ep + o[p];
    out[DV.pb[p]] = ep - o[p];
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

// Rows 1, 9, 11, 13, 14, 15 of Y(s)^T d, with S = Y(s) m^neq the Yu strain of Eq. LuoS at
// s_e = s1, s_nu = s (d = dJ/dS, off-diagonal components once).
struct YuT {
  float r1, r9, r11, r13, r14, r15;
};
__device__ __forceinline__ YuT yu_transpose(const float (&d)[6], float s1, float s, float ir) {
  YuT o;
  o.r1 = -s1 * ir * (1.0f / 38.0f) * (d[0] + d[1] + d[2]);
  o.r9 = s * ir * (-0.5f * d[0] + 0.25f * (d[1] + d[2]));
  o.r11 = s * ir * 0.75f * (d[2] - d[1]);
  o.r13 = -1.5f * s * ir * d[3];
  o.r14 = -1.5f * s * ir * d[4];
  o.r15 = -1.5f * s * ir * d[5];
  return o;
}

// (d m^eq / d j)^T y for y on rows 1, 9, 11, 13, 14, 15 (Eq. meq).
__device__ __forceinline__ void meq_j_transpose(const YuT& y, float jx, float jy, float jz, float ir, float& bx,
                                                float& by, float& bz) {
  bx = (38.0f * jx * y.r1 + 4.0f * jx * y.r9 + jy * y.r13 + jz * y.r15) * ir;
  by = (38.0f * jy * y.r1 - 2.0f * jy * y.r9 + 2.0f * jy * y.r11 + jx * y.r13 + jz * y.r14) * ir;
  bz = (38.0f * jz * y.r1 - 2.0f * jz * y.r9 - 2.0f * jz * y.r11 + jy * y.r14 + jx * y.r15) * ir;
}

// (dh/du)^T y on rows 1, 9, 11, 13, 14, 15 for h = S_F / 2, the half Guo source the
// force-corrected strain adds to the non-equilibrium moments. h is bilinear in u = j / rho0
// and F and symmetric in the two, so with a = F this is the derivative along u and with
// a = u the derivative along F.
__device__ __forceinline__ void half_source_transpose(const YuT& y, float ax, float ay, float az, float& ox, float& oy,
                                                      float& oz) {
  ox = 19.0f * ax * y.r1 + 2.0f * ax * y.r9 + 0.5f * (ay * y.r13 + az * y.r15);
  oy = 19.0f * ay * y.r1 - ay * y.r9 + ay * y.r11 + 0.5f * (ax * y.r13 + az * y.r14);
  oz = 19.0f * az * y.r1 - az * y.r9 - az * y.r11 + 0.5f * (ay * y.r14 + ax * y.r15);
}

// Strain S = P + s A from the six non-equilibrium moments of Eq. LuoS: P the s_e part, A the
// s_nu part at unit rate; gamma = |S| = sqrt(2 S:S) and dgamma/dS = 2 W S / gamma.
struct StrainParts {
  float A[6], S[6], dg[6], ss, gamma;
};
__device__ __forceinline__ StrainParts strain_parts(const float (&mn)[6], float s1, float s, float ir) {
  Neq n;
  n.m[1] = mn[0];
  n.m[9] = mn[1];
  n.m[11] = mn[2];
  n.m[13] = mn[3];
  n.m[14] = mn[4];
  n.m[15] = mn[5];
  StrainParts o;
  float P[6];
  strain_yu(n, s1, 0.0f, ir, P);
  strain_yu(n, 0.0f, 1.0f, ir, o.A);
#pragma unroll
  for (int c = 0; c < 6; ++c) o.S[c] = __builtin_fmaf(s, o.A[c], P[c]);
  o.ss = o.S[0] * o.S[0] + o.S[1] * o.S[1] + o.S[2] * o.S[2] +
         2.0f * (o.S[3] * o.S[3] + o.S[4] * o.S[4] + o.S[5] * o.S[5]);
  o.gamma = sqrtf(2.0f * o.ss);
  const float k = o.gamma > 0.0f ? 2.0f / o.gamma : 0.0f;
#pragma unroll
  for (int c = 0; c < 6; ++c) o.dg[c] = (c < 3 ? k : 2.0f * k) * o.S[c];
  return o;
}

// One reverse step. VISC: strain-dependent viscosity (kind 1, 2 lagged; 3 implicit), where
// the collision rate s_new depends on the state: the record of the forward step holds j,
// m^neq of rows 1, 9, 11, 13, 14, 15 and the strain's rate s_x; for the lagged kinds plane 19
// of lam_in / lam_out is the adjoint of the s_nu field (not streamed).
// IN_ROWS / OUT_ROWS: planes 0..18 of lam_in / lam_out in the row-interleaved order of the
// population buffers (element (i, z, y, x) at ((z ny + y) 19 + i) nx + x) instead of the
// canonical planes; a multi-step sweep keeps its intermediate states that way, so that
// a wave's 38 adjoint streams fall into the DRAM pages of a few rows. Plane 19 stays a plane
// (at 19 N) in both.
template <bool VISC, bool STAGE, bool IN_ROWS, bool OUT_ROWS>
__global__ __launch_bounds__(kMaxBlock) void adjoint_kernel(Geo G, ModelF M, ViscF V, ForceF Fo,
                                                            const float* __restrict__ rec,
                                                            const float* __restrict__ lam_in,
                                                            float* __restrict__ lam_out,
                                                            float* __restrict__ grad_force) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= G.nx || y >= G.ny) return;
  const Nbr ne = neighbours(G, x, y, z);
  const unsigned self = ne.self;
  const Nbr nb = in_bytes<float>(ne);
  const size_t N = G.N;
  Rows<Q, float> rows;
  if constexpr (IN_ROWS || OUT_ROWS) rows = rows_of<Q, float>(G, x, y, z);

  float lt[Q];
  if constexpr (IN_ROWS) {
    if constexpr (STAGE) pull_rows_staged<LatRev, float, true>(lam_in, G, rows, y, lt);
    else pull_rows<LatRev, float>(lam_in, G, rows, y, lt);
  } else {
    if constexpr (STAGE) pull_staged<LatRev, float, true>(lam_in, G, nb, y, lt);
    else pull<LatRev, float>(lam_in, G, nb, y, lt);
  }

  // mu = D^-1 T lam~
  const Pairs P = make_pairs(lt);
  float mu[Q];
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    mu[k] = moment<k>(P) * (1.0f / static_cast<float>(DV.D[k]));
  });

  const float jx = rec[self], jy = rec[N + self], jz = rec[2 * N + self];
  const float ir = M.inv_rho0;
  float snu = M.s[9];
  float mn[6], sx = 0.0f;
  StrainParts sp;
  if constexpr (VISC) {
#pragma unroll
    for (int c = 0; c < 6; ++c) mn[c] = rec[(3 + c) * N + self];
    sx = rec[9 * N + self];
    sp = strain_parts(mn, M.s[1], sx, ir);
    snu = V.kind == 3 ? sx : viscous_rate(sp.ss, V);
  }
  float w[Q], v[Q], nu[Q];
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    const float sk = is_nu_slot(k) ? snu : M.s[k];
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

  float gbx = 0.f, gby = 0.f, gbz = 0.f;  // extra dJ/dj through the rate
  float hfx = 0.f, hfy = 0.f, hfz = 0.f;  // extra dJ/dF through the force-corrected strain
  if constexpr (VISC) {
    // sensitivity of J to this collision's rate: dm*_k/ds = -(m^neq_k + S_F,k / 2) on the
    // s_nu rows, plus the adjoint of the s_nu field this collision writes (lagged kinds).
    // With the force-corrected strain the record already holds m^neq + S_F / 2.
    float SF9 = 0.f, SF11 = 0.f, SF13 = 0.f, SF14 = 0.f, SF15 = 0.f;
    if (Fo.mode && !Fo.strain_corr) {
      SF9 = (4.0f * jx * Fx - 2.0f * jy * Fy - 2.0f * jz * Fz) * ir;
      SF11 = (2.0f * jy * Fy - 2.0f * jz * Fz) * ir;
      SF13 = (jx * Fy + jy * Fx) * ir;
      SF14 = (jy * Fz + jz * Fy) * ir;
      SF15 = (jx * Fz + jz * Fx) * ir;
    }
    float sigma = -(mu[9] * (mn[1] + 0.5f * SF9) + mu[11] * (mn[2] + 0.5f * SF11) + mu[13] * (mn[3] + 0.5f * SF13) +
                    mu[14] * (mn[4] + 0.5f * SF14) + mu[15] * (mn[5] + 0.5f * SF15));
    const bool lagged = V.kind != 3;
    if (lagged) sigma += lam_in[19 * N + self];
    float dA = 0.f;
#pragma unroll
    for (int c = 0; c < 6; ++c) dA += sp.dg[c] * sp.A[c];
    float cg;  // dJ/dgamma through the rate
    if (lagged) {
      cg = sigma * (-3.0f * viscous_slope(sp.gamma, V) * snu * snu);
    } else {
      const float c0 = 3.0f * V.nu0 + 0.5f, k = 3.0f * V.csmag2;
      cg = -sigma * snu * k / (c0 + k * sp.gamma + snu * k * dA);
    }
    float d6[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) d6[c] = cg * sp.dg[c];
    if (lagged) lam_out[19 * N + self] = cg * dA;
    // dJ/dm^neq = Y(s_x)^T d6; m^neq = m - m^eq(drho, j): (I - E)^T on it
    const YuT yv = yu_transpose(d6, M.s[1], sx, ir);
    meq_j_transpose(yv, jx, jy, jz, ir, gbx, gby, gbz);
    if (Fo.strain_corr) {
      // the strain's input also holds h(j, F) = S_F / 2
      float hx, hy, hz;
      half_source_transpose(yv, Fx, Fy, Fz, hx, hy, hz);
      gbx -= hx * ir;
      gby -= hy * ir;
      gbz -= hz * ir;
      half_source_transpose(yv, jx * ir, jy * ir, jz * ir, hfx, hfy, hfz);
    }
    nu[0] += 11.0f * yv.r1;
    nu[1] += yv.r1;
    nu[9] += yv.r9;
    nu[11] += yv.r11;
    nu[13] += yv.r13;
    nu[14] += yv.r14;
    nu[15] += yv.r15;
    nu[3] -= gbx;
    nu[5] -= gby;
    nu[7] -= gbz;
  }

  float lo[Q];
  apply_transpose(nu, lo);
  if constexpr (OUT_ROWS) store_rows<Q, float>(lam_out, G, rows, lo);
  else store_local<Q>(lam_out, G, nb.self, lo);

  if (grad_force) {
    // G(j) = d S_F / d F
    const float Cx = (38.0f * jx * v[1] - 11.0f * jx * v[2] + 4.0f * jx * v[9] - 2.0f * jx * v[10] + jy * v[13] +
                      jz * v[15]) * ir + v[3] - (2.0f / 3.0f) * v[4];
    const float Cy = (38.0f * jy * v[1] - 11.0f * jy * v[2] - 2.0f * jy * v[9] + jy * v[10] + 2.0f * jy * v[11] -
                      jy * v[12] + jx * v[13] + jz * v[14]) * ir + v[5] - (2.0f / 3.0f) * v[6];
    const float Cz = (38.0f * jz * v[1] - 11.0f * jz * v[2] - 2.0f * jz * v[9] + jz * v[10] - 2.0f * jz * v[11] +
                      jz * v[12] + jy * v[14] + jx * v[15]) * ir + v[7] - (2.0f / 3.0f) * v[8];
    grad_force[self] += 0.5f * (Ax + Bx - gbx) + Cx + hfx;
    grad_force[N + self] += 0.5f * (Ay + By - gby) + Cy + hfy;
    grad_force[2 * N + self] += 0.5f * (Az + Bz - gbz) + Cz + hfz;
  }
}

// Loss J = sum_x S:S (Yu strain of the current pre-collision state, at the rate the model
// gives it: s_nu of p, the lagged field, or the implicitly solved rate) and its gradients.
// For the lagged kinds plane 19 of lam_out receives dJ/d(s_nu field).
template <typename S>
__global__ __launch_bounds__(256) void loss_seed_kernel(Geo G, ModelF M, ViscF V, ForceF Fo, const S* __restrict__ buf,
                                                        const float* __restrict__ snu_f, float* __restrict__ lam_out,
                                                        float* __restrict__ grad_force, double* __restrict__ partials) {
  double acc[kReduceVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  // blocks take whole x-rows in turn; the threads of a block walk along the row
  const unsigned rows = static_cast<unsigned>(G.ny) * G.nz;
  for (unsigned r = blockIdx.x; r < rows; r += gridDim.x) {
    const int y = r % G.ny;
    const int z = r / G.ny;
    for (int x = threadIdx.x; x < G.nx; x += blockDim.x) {
      const Node<Q, S> nb = node_at<Q, S>(G, x, y, z);
      const unsigned self = nb.self;
      float g[Q];
      pull_rows<LatFwd, S>(buf, G, nb.rows, y, g);
      const Pairs P = make_pairs(g);
      const float drho = delta_rho(P);
      float Fx, Fy, Fz;
      force_at(Fo, G.N, self, Fx, Fy, Fz);
      const float jx = momentum<0>(P) + 0.5f * Fx, jy = momentum<1>(P) + 0.5f * Fy, jz = momentum<2>(P) + 0.5f * Fz;
      Neq n = noneq_moments(P, drho, jx, jy, jz, M);
      const float s1 = M.s[1], ir = M.inv_rho0;
      if (Fo.strain_corr) {
        // force-corrected strain: the moments the strain takes include S_F / 2
        float SF[Q];
        force_moments(jx, jy, jz, Fx, Fy, Fz, ir, SF);
        n.m[1] += 0.5f * SF[1];
        n.m[9] += 0.5f * SF[9];
        n.m[11] += 0.5f * SF[11];
        n.m[13] += 0.5f * SF[13];
        n.m[14] += 0.5f * SF[14];
        n.m[15] += 0.5f * SF[15];
      }
      float sn = M.s[9];
      if (V.kind == 3) sn = implicit_rate_yu(n, M, V);
      else if (V.kind != 0) sn = snu_f[self];
      const float mn[6] = {n.m[1], n.m[9], n.m[11], n.m[13], n.m[14], n.m[15]};
      const StrainParts sp = strain_parts(mn, s1, sn, ir);
      const float* S6 = sp.S;
      acc[0] += static_cast<double>(S6[0]) * S6[0] + static_cast<double>(S6[1]) * S6[1] +
                static_cast<double>(S6[2]) * S6[2] +
                2.0 * (static_cast<double>(S6[3]) * S6[3] + static_cast<double>(S6[4]) * S6[4] +
                       static_cast<double>(S6[5]) * S6[5]);
      // dJ/dS = 2 W S, and dJ/ds = (2 W S) . A at the strain's rate
      float d6[6] = {2.0f * S6[0], 2.0f * S6[1], 2.0f * S6[2], 4.0f * S6[3], 4.0f * S6[4], 4.0f * S6[5]};
      float dJds = 0.f;
#pragma unroll
      for (int c = 0; c < 6; ++c) dJds += d6[c] * sp.A[c];
      if (V.kind == 3) {
        // the implicit rate moves with the state: ds/dm^neq = -k s (dgamma/dS)^T Y(s) / dG/ds
        float dA = 0.f;
#pragma unroll
        for (int c = 0; c < 6; ++c) dA += sp.dg[c] * sp.A[c];
        const float c0 = 3.0f * V.nu0 + 0.5f, k = 3.0f * V.csmag2;
        const float cg = -dJds * sn * k / (c0 + k * sp.gamma + sn * k * dA);
#pragma unroll
        for (int c = 0; c < 6; ++c) d6[c] = __builtin_fmaf(cg, sp.dg[c], d6[c]);
      } else if (V.kind != 0) {
        lam_out[19 * static_cast<size_t>(G.N) + self] = dJds;
      }
      // sigma = Y(s)^T dJ/dS on rows 1, 9, 11, 13..15 of m^neq
      const YuT yv = yu_transpose(d6, s1, sn, ir);
      float sg[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) sg[k] = 0.0f;
      sg[1] = yv.r1;
      sg[9] = yv.r9;
      sg[11] = yv.r11;
      sg[13] = yv.r13;
      sg[14] = yv.r14;
      sg[15] = yv.r15;
      // lam = T^T sigma - (dm^eq/dg)^T sigma,  (dm^eq/dg)^T sigma = a 1 + C^T b
      float lam[Q];
      apply_transpose(sg, lam);
      const float a = -11.0f * sg[1];
      float bx, by, bz, hfx = 0.f, hfy = 0.f, hfz = 0.f;
      meq_j_transpose(yv, jx, jy, jz, ir, bx, by, bz);
      if (Fo.strain_corr) {
        float hx, hy, hz;
        half_source_transpose(yv, Fx, Fy, Fz, hx, hy, hz);
        bx -= hx * ir;
        by -= hy * ir;
        bz -= hz * ir;
        half_source_transpose(yv, jx * ir, jy * ir, jz * ir, hfx, hfy, hfz);
      }
      static_for<Q>([&](auto ii) {
        constexpr int i = ii;
        lam[i] -= a + static_cast<float>(CX[i]) * bx + static_cast<float>(CY[i]) * by + static_cast<float>(CZ[i]) * bz;
      });
      store_local<Q>(lam_out, G, self * 4u, lam);
      if (grad_force) {
        grad_force[self] += hfx - 0.5f * bx;
        grad_force[G.N + self] += hfy - 0.5f * by;
        grad_force[2 * static_cast<size_t>(G.N) + self] += hfz - 0.5f * bz;
      }
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

template <bool IN_ROWS, bool OUT_ROWS>
static hipError_t launch_adjoint_layout(const Geo& G, const ModelF& M, const ViscF& V, const ForceF& Fo,
                                        const float* rec, const float* lam_in, float* lam_out, float* grad_force,
                                        hipStream_t st) {
  const Launch L = node_launch(G);
  // whole-row blocks exchange the x-shifted adjoint elements through LDS (pull_mode 2)
  const bool stage = pull_mode(G, L.block) == 2;
  if (V.kind == 0) {
    // constant viscosity, whole 256-node rows: 6 blocks per CU instead of 7 (+2.5 % at 256^3;
    // 4 blocks lost 4 %; the 128^3 shape and the lagged kernel run as fast uncapped)
    const size_t lds = (stage && L.block.x == 256) ? lds_cap_bytes(6, staged_lds_bytes<LatRev>()) : 0;
    if (stage)
      hipLaunchKernelGGL((adjoint_kernel<false, true, IN_ROWS, OUT_ROWS>), L.grid, L.block, lds, st, G, M, V, Fo, rec,
                         lam_in, lam_out, grad_force);
    else
      hipLaunchKernelGGL((adjoint_kernel<false, false, IN_ROWS, OUT_ROWS>), L.grid, L.block, 0, st, G, M, V, Fo, rec,
                         lam_in, lam_out, grad_force);
  } else {
    if (stage)
      hipLaunchKernelGGL((adjoint_kernel<true, true, IN_ROWS, OUT_ROWS>), L.grid, L.block, 0, st, G, M, V, Fo, rec,
                         lam_in, lam_out, grad_force);
    else
      hipLaunchKernelGGL((adjoint_kernel<true, false, IN_ROWS, OUT_ROWS>), L.grid, L.block, 0, st, G, M, V, Fo, rec,
                         lam_in, lam_out, grad_force);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_step(const Geo& G, const ModelF& M, const ViscF& V, const ForceF& Fo, const float* rec,
                               const float* lam_in, float* lam_out, float* grad_force, hipStream_t st, bool in_rows,
                               bool out_rows) {
  if (in_rows) {
    if (out_rows) return launch_adjoint_layout<true, true>(G, M, V, Fo, rec, lam_in, lam_out, grad_force, st);
    return launch_adjoint_layout<true, false>(G, M, V, Fo, rec, lam_in, lam_out, grad_force, st);
  }
  if (out_rows) return launch_adjoint_layout<false, true>(G, M, V, Fo, rec, lam_in, lam_out, grad_force, st);
  return launch_adjoint_layout<false, false>(G, M, V, Fo, rec, lam_in, lam_out, grad_force, st);
}

hipError_t launch_loss_seed(int storage, const Geo& G, const ModelF& M, const ViscF& V, const ForceF& Fo,
                            const void* buf, const float* snu, float* lam_out, float* grad_force, double* partials,
                            double* out, hipStream_t st) {
  unsigned nb = static_cast<unsigned>(G.ny) * G.nz;  // one x-row per block at a time
  if (nb > static_cast<unsigned>(kReduceBlocks)) nb = kReduceBlocks;
  switch (storage) {
    case 0: hipLaunchKernelGGL(loss_seed_kernel<float>, dim3(nb), dim3(256), 0, st, G, M, V, Fo, static_cast<const float*>(buf), snu, lam_out, grad_force, partials); break;
    case 1: hipLaunchKernelGGL(loss_seed_kernel<_Float16>, dim3(nb), dim3(256), 0, st, G, M, V, Fo, static_cast<const _Float16*>(buf), snu, lam_out, grad_force, partials); break;
    case 2: hipLaunchKernelGGL(loss_seed_kernel<__bf16>, dim3(nb), dim3(256), 0, st, G, M, V, Fo, static_cast<const __bf16*>(buf), snu, lam_out, grad_force, partials); break;
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
