// D2Q9 kernels: the same fused pull-stream / collide / strain step as D3Q19 on the
// nine-velocity lattice (Sections 5.3 and 5.4 of the paper), plus initial state, strain
// query, canonical gather/scatter and the diagnostics reduction. One thread per node.
#include <hip/hip_runtime.h>

// Contraction of a product and a sum into an FMA only within one expression of the source
// (for this file and the headers it includes): left to the code generator, which product of
// a sum gets fused depends on the code around it, and the two-step kernel below must round
// every operation as the single step does.
#pragma clang fp contract(on)

#include "d2q9.h"
#include "internal.h"
#include "launch.h"
#include "reduce.h"

namespace lbm {
namespace d2q9 {

__device__ __forceinline__ void load_force(const ForceF& Fo, unsigned N, unsigned self, float& Fx, float& Fy) {
  if (Fo.mode == 1) {
    Fx = Fo.F[0];
    Fy = Fo.F[1];
  } else if (Fo.mode == 2) {
    Fx = Fo.field[self];
    Fy = Fo.field[N + self];
  } else {
    Fx = Fy = 0.0f;
  }
}

__device__ __forceinline__ void rates_with(const ModelF& M, float snu, float (&r)[Q]) {
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    r[k] = is_nu_slot(k) ? snu : M.s[k];
  });
}

// S:S (the off-diagonal component counts twice) in one fixed order of operations. Written as
// plain products and sums, the compiler may fuse either product of a sum into an FMA, and
// which one it picks depends on the code around it, so the same strain could round to two
// different rates in two kernels; the two-step kernel must round exactly as the single step.
__device__ __forceinline__ float strain_sq(const float (&S)[3]) {
  return __builtin_fmaf(S[0], S[0], __builtin_fmaf(S[1], S[1], 2.0f * S[2] * S[2]));
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
__device__ __forceinline__ StrainIn<true> strain_in_state(const Neq& n, float jx, float jy, float Fx, float Fy,
                                                          const ModelF& M, const ForceF& Fo) {
  float SF[Q];
  if (Fo.strain_corr) {
    force_moments(jx, jy, Fx, Fy, M.inv_rho0, SF);
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) SF[k] = 0.0f;
  }
  return strain_in<true>(n, SF);
}

template <bool CORR>
__device__ __forceinline__ void strain_chai_in(const Pairs& P, float drho, float jx, float jy, const float (&rates)[Q],
                                               const StrainIn<CORR>& si, float inv_rho0, float (&S)[3]) {
  strain_chai(P, drho, jx, jy, rates, inv_rho0, S);
  if constexpr (CORR) {
    float Sh[3];
    strain_yu(si.h, rates[1], rates[7], inv_rho0, Sh);
#pragma unroll
    for (int c = 0; c < 3; ++c) S[c] += Sh[c];
  }
}

// s_nu of the implicit Smagorinsky coupling at one node, from the formula V selects (both
// are affine in s_nu: split into the part at the other rates and the s_nu rows).
template <bool CORR>
__device__ __forceinline__ float implicit_rate(const Pairs& P_, float drho, float jx, float jy,
                                               const StrainIn<CORR>& si, const ModelF& M, const ViscF& V) {
  float P[3], A[3];
  if (V.drive_chai) {
    float rb[Q], rn[Q];
    rates_with(M, 0.0f, rb);
    static_for<Q>([&](auto ki) {
      constexpr int k = ki;
      rn[k] = is_nu_slot(k) ? 1.0f : 0.0f;
    });
    strain_chai_in(P_, drho, jx, jy, rb, si, M.inv_rho0, P);
    strain_chai_in(P_, drho, jx, jy, rn, si, M.inv_rho0, A);
  } else {
    strain_yu(si.ns, M.s[1], 0.0f, M.inv_rho0, P);
    strain_yu(si.ns, 0.0f, 1.0f, M.inv_rho0, A);
  }
  return implicit_smagorinsky(P, A, V.nu0, V.csmag2);
}

// The s_nu a strain query or the diagnostics take the strain with: the stored lagged rate,
// the implicit rate of the state itself, or the constant rate.
__device__ __forceinline__ float query_rate(const Pairs& P, float drho, float jx, float jy, const StrainIn<true>& si,
                                            const ModelF& M, const ViscF& V, const float* snu_f, unsigned self) {
  if (V.kind == 3) return implicit_rate(P, drho, jx, jy, si, M, V);
  return snu_f ? snu_f[self] : M.s[7];
}

// One node's collision with its strain and viscosity (Eq. mrteq's right side with the rates
// of Eq. mrteqvT; the strain of Section 5.3, or the Yu-type formula of Section 5.4): g holds
// the pulled populations on entry and the post-collision ones on return. lagged() gives the
// node's lagged rate (read only where the lagged coupling needs it), store_lagged(s) keeps
// the rate a lagged viscosity law derived for the next step. (Fx, Fy): the node's force
// (load_force). S_out / emit: the optional strain output (emit 1 Yu, 2 Chai). Returns the
// rate of s_nu's rows this collision used.
template <bool CORR, class Lagged, class StoreLagged>
__device__ __forceinline__ float collide(const Geo& G, const ModelF& M, const ViscF& V, const ForceF& Fo,
                                         unsigned self, Lagged lagged, StoreLagged store_lagged, float Fx, float Fy,
                                         float* S_out, int emit, float (&g)[Q]) {
  const Pairs P = make_pairs(g);
  const float drho = delta_rho(P);
  float jx = momentum<0>(P), jy = momentum<1>(P);
  if (Fo.mode) {
    jx = __builtin_fmaf(0.5f, Fx, jx);
    jy = __builtin_fmaf(0.5f, Fy, jy);
  }
  const Neq n = noneq_moments(P, drho, jx, jy, M.inv_rho0);
  // the Guo source in moment space; with CORR formed before the strain (half of it joins the
  // non-equilibrium part the strain takes)
  float SF[Q];
  if constexpr (CORR) force_moments(jx, jy, Fx, Fy, M.inv_rho0, SF);
  const StrainIn<CORR> si = strain_in<CORR>(n, SF);
  float Syu[3], Sch[3];
  float snu = M.s[7];
  if (V.kind == 3) {
    // implicit coupling: the strain at the rate of this very collision
    snu = implicit_rate(P, drho, jx, jy, si, M, V);
    if (S_out) {
      if (emit == 2) {
        float r[Q];
        rates_with(M, snu, r);
        strain_chai_in(P, drho, jx, jy, r, si, M.inv_rho0, Sch);
      } else {
        strain_yu(si.ns, M.s[1], snu, M.inv_rho0, Syu);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) stream_store(&S_out[static_cast<size_t>(c) * G.N + self], emit == 2 ? Sch[c] : Syu[c]);
    }
  } else {
    // lagged coupling: the strain of the incoming state with the rates of the previous collision
    const float snu_prev = lagged();
    const bool need_yu = emit == 1 || (V.kind != 0 && !V.drive_chai);
    const bool need_chai = emit == 2 || (V.kind != 0 && V.drive_chai);
    if (need_yu) strain_yu(si.ns, M.s[1], snu_prev, M.inv_rho0, Syu);
    if (need_chai) {
      float r[Q];
      rates_with(M, snu_prev, r);
      strain_chai_in(P, drho, jx, jy, r, si, M.inv_rho0, Sch);
    }
    if (S_out) {
#pragma unroll
      for (int c = 0; c < 3; ++c) stream_store(&S_out[static_cast<size_t>(c) * G.N + self], emit == 2 ? Sch[c] : Syu[c]);
    }
    if (V.kind != 0) {
      snu = viscous_rate(V.drive_chai ? strain_sq(Sch) : strain_sq(Syu), V);
      store_lagged(snu);
    }
  }
  float dm[Q];
  dm[0] = 0.0f;
  dm[3] = Fx;
  dm[5] = Fy;
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    if constexpr (k != 0 && k != 3 && k != 5) dm[k] = -(is_nu_slot(k) ? snu : M.s[k]) * n.m[k];
  });
  if (Fo.mode) {
    if constexpr (!CORR) force_moments(jx, jy, Fx, Fy, M.inv_rho0, SF);
    static_for<Q>([&](auto ki) {
      constexpr int k = ki;
      if constexpr (k != 0 && k != 3 && k != 5) {
        const float sk = is_nu_slot(k) ? snu : M.s[k];
        dm[k] = __builtin_fmaf(1.0f - 0.5f * sk, SF[k], dm[k]);
      }
    });
  }
  add_back_transform(dm, g);
  return snu;
}

// XMODE: how a block pulls along x (pull_mode: 0 part rows, 1 whole rows, 2 whole rows with
// the LDS exchange). CORR: the force-corrected strain (a separate instance, so that the plain
// step keeps its register budget).
template <typename S, bool WALLS, int XMODE, bool CORR>
__global__ __launch_bounds__(kMaxBlock) void step_kernel(Geo G, ModelF M, ViscF V, ForceF Fo, StepIO io) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const unsigned self = node_index(G, x, y, 0);
  const Rows<Q, S> r = rows_of<Q, S>(G, x, y, 0);
  float g[Q];
  if constexpr (XMODE == 2) pull_rows_staged<Lat, S, WALLS>(static_cast<const S*>(io.src), G, r, y, g);
  else pull_rows<Lat, S, WALLS, XMODE == 1>(static_cast<const S*>(io.src), G, r, y, g);
  float Fx, Fy;
  load_force(Fo, G.N, self, Fx, Fy);
  collide<CORR>(
      G, M, V, Fo, self, [&] { return io.snu ? io.snu[self] : M.s[7]; }, [&](float s) { io.snu[self] = s; }, Fx,
      Fy, io.S_out, io.emit, g);
  store_rows<Q>(static_cast<S*>(io.dst), G, r, g);
}

// Two steps per launch: the
// result is that of two launches of step_kernel, bit for bit, for the algorithmic HBM
// traffic of one (the rows at block edges are read twice).
// A block of 256 lanes owns a strip of kPairStrip columns (lane l at column x0 - 1 + l, the
// two edge lanes a ring column on either side, wrapped periodically) and kPairRows rows of
// the result, and walks its rows upwards. At row t it pulls the incoming state from HBM and
// collides it (level 1, rounded to the storage type as a store would round it); the
// populations a neighbouring lane pulls at level 2 (c_x != 0) go to an LDS ring of rows,
// those the lane itself pulls (c_x = 0) stay in registers. After one barrier it pulls row
// t - 1 of level 1 (from rows t - 2, t - 1 and t), collides it again and stores it. The ring
// is deep enough that one barrier per row suffices: the slot written at row t + 1 is none of
// those read at row t. Level 1 is computed for the two ring columns and for
// one extra row below and above the block's rows, as the neighbouring blocks compute them
// too: 256 / 254 more columns and (kPairRows + 2) / kPairRows more rows of level-1 work.
// The lagged rate s_nu cannot be updated in place (a neighbour still reads the old value of
// a ring node after this block has passed it), so it is read from snu_in and written to
// snu_out.
constexpr int kPairStrip = 254;
// Rows per block: fewer rows mean more level-1 rows computed twice, more rows fewer blocks
// to overlap one another's barriers and memory waits. Measured at 4096^2: FP32 105.6k MLUPS
// at 6 rows, 102.9k at 8 and 103.8k at 12; FP16 156.5k, 159.4k and 159.8k.
template <typename S>
constexpr int kPairRows = sizeof(S) == 4 ? 6 : 12;

// LDS ring rows of the x-shifted populations: one with c_y = -1 is read in the row it was
// written (2 slots: a fast thread writes the next row while a slow one still reads this one),
// the others one or two rows later (4 slots); ring_row(i) is population i's first slot. With
// walls a population is also read one row later as the opposite of one that bounces back:
// 4 slots for all.
template <bool WALLS>
constexpr int ring_rows(int i) { return Lat::cx(i) == 0 ? 0 : (Lat::cy(i) < 0 && !WALLS ? 2 : 4); }
template <bool WALLS>
constexpr int ring_row(int i) { return i == 0 ? 0 : ring_row<WALLS>(i - 1) + ring_rows<WALLS>(i - 1); }

// WALLS: halfway bounce-back at y = -1/2 and ny - 1/2 (no wrap in y; level 1 is not computed
// for the rows beyond the walls, and a population of level 2 that crosses a wall is the
// opposite one of the node's own level-1 state). CORR: the force-corrected strain.
// EMIT: the strain output S_out (emit 1 Yu, 2 Chai), taken at level 2 only (the strain of
// the second step's incoming state, which single steps leave in S_out last); a template
// parameter, as its code costs the instances without it 15 VGPRs otherwise.
template <typename S, bool WALLS, bool CORR, bool EMIT>
__global__ __launch_bounds__(256) void pair_kernel(Geo G, ModelF M, ViscF V, ForceF Fo, const S* __restrict__ src,
                                                   S* __restrict__ dst, const float* snu_in, float* snu_out,
                                                   float* S_out, int emit) {
  // (in the storage type: level 1 is rounded to it anyway, and 16-bit rows halve the LDS)
  __shared__ S ring[ring_row<WALLS>(Q)][256];
  const int lane = threadIdx.x;
  const int x0 = blockIdx.x * kPairStrip;
  const int xl = x0 - 1 + lane;  // this lane's column, unwrapped
  // (nx >= 256, so that every lane's column wraps into the box: lanes past the ring column
  // of a ragged last strip compute level 1 of a column no one reads, and every lane takes
  // the same path through level 1)
  const int x = xl < 0 ? xl + G.nx : (xl >= G.nx ? xl - G.nx : xl);
  const bool kept = lane >= 1 && lane <= kPairStrip && xl < G.nx;  // level 2 owned here
  const int y0 = blockIdx.y * kPairRows<S>;
  const int rows = min(kPairRows<S>, G.ny - y0);
  // level-1 values of the c_x = 0 populations this lane pulls back one and two rows later
  float prev[Q], prev2[Q], snu_prev = 0.0f;
  constexpr auto slot = [](int i, int row) { return ring_row<WALLS>(i) + (row & (ring_rows<WALLS>(i) - 1)); };
  for (int k = 0; k < rows + 2; ++k) {
    int t = y0 - 1 + k;
    float g[Q], snu1 = 0.0f;
    if (!WALLS) t = t < 0 ? t + G.ny : (t >= G.ny ? t - G.ny : t);
    if (!WALLS || (t >= 0 && t < G.ny)) {  // (uniform over the block)
      pull_rows<Lat, S, WALLS, false>(src, G, rows_of<Q, S>(G, x, t, 0), t, g);
      const unsigned self1 = node_index(G, x, t, 0);
      float Fx, Fy;
      load_force(Fo, G.N, self1, Fx, Fy);
      snu1 = collide<CORR>(
          G, M, V, Fo, self1, [&] { return snu_in ? snu_in[self1] : M.s[7]; }, [](float) {}, Fx, Fy, nullptr, 0, g);
      static_for<Q>([&](auto ii) {
        constexpr int i = ii;
        if constexpr (sizeof(S) == 2) g[i] = static_cast<float>(static_cast<S>(g[i]));
        // opaque: no operation of level 2 may be fused with the last one of level 1
        asm volatile("" : "+v"(g[i]));
        if constexpr (Lat::cx(i) != 0) ring[slot(i, k)][lane] = static_cast<S>(g[i]);
      });
      asm volatile("" : "+v"(snu1));
    } else {
      static_for<Q>([&](auto ii) { g[ii] = 0.0f; });  // a row beyond a wall: never pulled
    }
    __syncthreads();
    if (k >= 2 && kept) {
      const int y = y0 + k - 2;
      float h[Q];
      static_for<Q>([&](auto ii) {
        constexpr int i = ii;
        constexpr int cx = Lat::cx(i), cy = Lat::cy(i), o = Lat::opp(i);
        float v;
        if constexpr (cx != 0) v = static_cast<float>(ring[slot(i, k - 1 - cy)][lane - cx]);
        else if constexpr (cy == 0) v = prev[i];
        else if constexpr (cy > 0) v = prev2[i];
        else v = g[i];
        if constexpr (WALLS && cy != 0) {
          // bounce-back: the opposite population of this node's own level-1 state (row k - 1)
          float b;
          if constexpr (Lat::cx(o) != 0) b = static_cast<float>(ring[slot(o, k - 1)][lane]);
          else b = prev[o];
          if (crosses_wall<cy>(G, y)) v = b;
        }
        h[i] = v;
      });
      const unsigned self = node_index(G, x, y, 0);
      float Fx, Fy;
      load_force(Fo, G.N, self, Fx, Fy);
      collide<CORR>(
          G, M, V, Fo, self, [&] { return snu_prev; }, [&](float s) { snu_out[self] = s; }, Fx, Fy,
          EMIT ? S_out : nullptr, EMIT ? emit : 0, h);
      store_rows<Q>(dst, G, rows_of<Q, S>(G, x, y, 0), h);
    }
    static_for<Q>([&](auto ii) {
      constexpr int i = ii;
      if constexpr (Lat::cx(i) == 0) {
        prev2[i] = prev[i];
        prev[i] = g[i];
      }
    });
    snu_prev = snu1;
  }
}

template <typename S>
__global__ __launch_bounds__(kMaxBlock) void strain_kernel(Geo G, ModelF M, ViscF V, ForceF Fo, const S* buf,
                                                           const float* snu_f, int kind, float* S_out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const Node<Q, S> nb = node_at<Q, S>(G, x, y, 0);
  float g[Q];
  pull_rows<Lat, S>(buf, G, nb.rows, y, g);
  const Pairs P = make_pairs(g);
  const float drho = delta_rho(P);
  float Fx, Fy;
  load_force(Fo, G.N, nb.self, Fx, Fy);
  const float jx = momentum<0>(P) + 0.5f * Fx, jy = momentum<1>(P) + 0.5f * Fy;
  const Neq n = noneq_moments(P, drho, jx, jy, M.inv_rho0);
  const StrainIn<true> si = strain_in_state(n, jx, jy, Fx, Fy, M, Fo);
  const float snu = query_rate(P, drho, jx, jy, si, M, V, snu_f, nb.self);
  float S3[3];
  if (kind == 2) {
    float r[Q];
    rates_with(M, snu, r);
    strain_chai_in(P, drho, jx, jy, r, si, M.inv_rho0, S3);
  } else {
    strain_yu(si.ns, M.s[1], snu, M.inv_rho0, S3);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) stream_store(&S_out[static_cast<size_t>(c) * G.N + nb.self], S3[c]);
}

template <typename S>
__global__ __launch_bounds__(kMaxBlock) void init_kernel(Geo G, ModelF M, S* buf, float* snu, const float* rho_u,
                                                   const float* grad_u) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const Node<Q, S> nb = node_at<Q, S>(G, x, y, 0);
  const unsigned self = nb.self;
  float drho = 0.f, ux = 0.f, uy = 0.f;
  if (rho_u) {
    drho = rho_u[self];
    ux = rho_u[G.N + self];
    uy = rho_u[2 * static_cast<size_t>(G.N) + self];
  }
  float g[Q];
  equilibrium(drho, M.rho0 * ux, M.rho0 * uy, M.inv_rho0, g);
  if (grad_u) {
    // d[a*3+b] = d j_b / d x_a; inverse of the Yu-type formula (Chapman-Enskog state).
    const size_t N = G.N;
    const float dxx = M.rho0 * grad_u[0 * N + self], dxy = M.rho0 * grad_u[1 * N + self];
    const float dyx = M.rho0 * grad_u[3 * N + self], dyy = M.rho0 * grad_u[4 * N + self];
    const float sn = M.s[7];
    float mn[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) mn[k] = 0.0f;
    mn[1] = -2.0f * (dxx + dyy) / M.s[1];
    mn[7] = -2.0f * (dxx - dyy) / (3.0f * sn);
    mn[8] = -(dxy + dyx) / (3.0f * sn);
    add_back_transform(mn, g);
  }
  scatter_rows<Lat, S>(buf, G, nb.rows, y, g);
  if (snu) snu[self] = M.s[7];
}

template <typename S>
__global__ __launch_bounds__(kMaxBlock) void get_kernel(Geo G, const S* buf, float* canon) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const Node<Q, S> nb = node_at<Q, S>(G, x, y, 0);
  float g[Q];
  pull_rows<Lat, S>(buf, G, nb.rows, y, g);
  store_local<Q>(canon, G, nb.self * 4u, g);
}

template <typename S>
__global__ __launch_bounds__(kMaxBlock) void set_kernel(Geo G, S* buf, const float* canon) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const Node<Q, S> nb = node_at<Q, S>(G, x, y, 0);
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
  for (int y = blockIdx.x; y < G.ny; y += gridDim.x) {
    for (int x = threadIdx.x; x < G.nx; x += blockDim.x) {
      const Node<Q, S> nb = node_at<Q, S>(G, x, y, 0);
      float g[Q];
      pull_rows<Lat, S>(buf, G, nb.rows, y, g);
      int bad = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) bad += !isfinite(g[i]);
      const Pairs P = make_pairs(g);
      const float drho = delta_rho(P);
      float Fx, Fy;
      load_force(Fo, G.N, nb.self, Fx, Fy);
      const float jx = momentum<0>(P) + 0.5f * Fx, jy = momentum<1>(P) + 0.5f * Fy;
      const Neq n = noneq_moments(P, drho, jx, jy, M.inv_rho0);
      float S3[3];
      const StrainIn<true> si = strain_in_state(n, jx, jy, Fx, Fy, M, Fo);
      strain_yu(si.ns, M.s[1], query_rate(P, drho, jx, jy, si, M, V, snu_f, nb.self), M.inv_rho0, S3);
      const double jj = static_cast<double>(jx) * jx + static_cast<double>(jy) * jy;
      acc[0] += drho;
      acc[1] += jx;
      acc[2] += jy;
      acc[4] += jj * (0.5 / M.rho0);
      acc[5] += static_cast<double>(S3[0]) * S3[0] + static_cast<double>(S3[1]) * S3[1] +
                2.0 * static_cast<double>(S3[2]) * S3[2];
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
  switch (pull_mode(G, L.block) + (walls ? 3 : 0)) {
    case 0: hipLaunchKernelGGL((step_kernel<S, false, 0, CORR>), L.grid, L.block, 0, st, G, M, V, Fo, io); break;
    case 1: hipLaunchKernelGGL((step_kernel<S, false, 1, CORR>), L.grid, L.block, 0, st, G, M, V, Fo, io); break;
    case 2: hipLaunchKernelGGL((step_kernel<S, false, 2, CORR>), L.grid, L.block, 0, st, G, M, V, Fo, io); break;
    case 3: hipLaunchKernelGGL((step_kernel<S, true, 0, CORR>), L.grid, L.block, 0, st, G, M, V, Fo, io); break;
    case 4: hipLaunchKernelGGL((step_kernel<S, true, 1, CORR>), L.grid, L.block, 0, st, G, M, V, Fo, io); break;
    default: hipLaunchKernelGGL((step_kernel<S, true, 2, CORR>), L.grid, L.block, 0, st, G, M, V, Fo, io); break;
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

template <typename S, bool W, bool C, bool E>
static void launch_pair_k(const dim3& grid, hipStream_t st, const Geo& G, const ModelF& M, const ViscF& V,
                          const ForceF& Fo, const void* src, void* dst, const float* snu_in, float* snu_out,
                          float* S_out, int emit) {
  hipLaunchKernelGGL((pair_kernel<S, W, C, E>), grid, dim3(256), 0, st, G, M, V, Fo, cb<S>(src), static_cast<S*>(dst),
                     snu_in, snu_out, S_out, emit);
}

template <typename S>
static void launch_pair_s(unsigned strips, hipStream_t st, const Geo& G, const ModelF& M, const ViscF& V,
                          const ForceF& Fo, const void* src, void* dst, const float* snu_in, float* snu_out,
                          float* S_out, int emit) {
  const dim3 grid(strips, (G.ny + kPairRows<S> - 1) / kPairRows<S>, 1);
  decltype(&launch_pair_k<S, false, false, false>) k;
  switch ((G.walls ? 1 : 0) + (Fo.strain_corr ? 2 : 0) + (S_out ? 4 : 0)) {
    case 0: k = launch_pair_k<S, false, false, false>; break;
    case 1: k = launch_pair_k<S, true, false, false>; break;
    case 2: k = launch_pair_k<S, false, true, false>; break;
    case 3: k = launch_pair_k<S, true, true, false>; break;
    case 4: k = launch_pair_k<S, false, false, true>; break;
    case 5: k = launch_pair_k<S, true, false, true>; break;
    case 6: k = launch_pair_k<S, false, true, true>; break;
    default: k = launch_pair_k<S, true, true, true>; break;
  }
  k(grid, st, G, M, V, Fo, src, dst, snu_in, snu_out, S_out, emit);
}

bool pair_supported(const Geo& G) {
  // (narrower boxes leave most lanes of a strip idle; the grid's y extent is at most 65535)
  return G.nz == 1 && G.nx >= 256 && (G.ny + 5) / 6 <= 65535;
}

hipError_t launch_pair(int storage, const Geo& G, const ModelF& M, const ViscF& V, const ForceF& Fo, const void* src,
                       void* dst, const float* snu_in, float* snu_out, float* S_out, int emit, hipStream_t st) {
  if (!pair_supported(G)) return hipErrorInvalidValue;
  if ((V.kind == 1 || V.kind == 2) != (snu_in != nullptr) || (snu_in != nullptr) != (snu_out != nullptr) ||
      (snu_in && snu_in == snu_out))
    return hipErrorInvalidValue;
  const unsigned strips = (G.nx + kPairStrip - 1) / kPairStrip;
  switch (storage) {
    case 0: launch_pair_s<float>(strips, st, G, M, V, Fo, src, dst, snu_in, snu_out, S_out, emit); break;
    case 1: launch_pair_s<_Float16>(strips, st, G, M, V, Fo, src, dst, snu_in, snu_out, S_out, emit); break;
    case 2: launch_pair_s<__bf16>(strips, st, G, M, V, Fo, src, dst, snu_in, snu_out, S_out, emit); break;
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
  unsigned nb = static_cast<unsigned>(G.ny);  // one x-row per block at a time
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

}  // namespace d2q9
}  // namespace lbm
