// D3Q19 fused collide-stream-strain step.
//
// One thread owns one node. The step pulls the 19 post-collision populations of the
// previous step from the neighbours (Eq. mrteq read backwards), forms the moments
// m = T g (Section 2), the equilibrium moments (Eq. meq), the strain of this pre-collision
// state by the Yu formula (Eq. LuoS) and/or the Chai formula (Eq. ChaiS), the new s_nu of
// the viscosity model, relaxes in moment space (Eq. mrteqvT) and stores the 19
// post-collision populations at the node itself. Loads are coalesced along x (shifted by
// at most one element), stores are aligned and coalesced.
#include <hip/hip_runtime.h>

#include "d3q19.h"
#include "d3q19_node.h"
#include "internal.h"
#include "launch.h"

namespace lbm {
namespace d3q19 {

// Everything one node does between the pull and the store: moments, strain of the incoming
// state (Yu and/or Chai, with the lagged s_nu or the implicitly solved one), viscosity
// model, relaxation with the Guo term, back-transform. g holds the pulled pre-collision
// populations on entry and the post-collision populations on exit; `self` is the node's
// element offset in the fields. PACK: g was converted from FP16 on load; the FP16 values are
// kept packed (pack_pairs) and both their uses, the pair sums and the final sums, read them
// through mixed-precision FMAs.
template <bool CORR, bool PACK>
__device__ __forceinline__ void node_update(float (&g)[Q], unsigned self, const Geo& G, const ModelF& M,
                                            const ViscF& V, const ForceF& Fo, const StepIO& io) {
  HalfPairs hp;
  Pairs P_;
  if constexpr (PACK) {
    hp = pack_pairs(g);
    P_ = make_pairs_packed(hp);
  } else {
    P_ = make_pairs(g);
  }
  const float drho = delta_rho(P_);
  float jx = momentum<0>(P_), jy = momentum<1>(P_), jz = momentum<2>(P_);
  float Fx, Fy, Fz;
  load_force(Fo, G.N, self, Fx, Fy, Fz);
  if (Fo.mode) {
    jx = __builtin_fmaf(0.5f, Fx, jx);
    jy = __builtin_fmaf(0.5f, Fy, jy);
    jz = __builtin_fmaf(0.5f, Fz, jz);
  }
  const Neq n = noneq_moments(P_, drho, jx, jy, jz, M);
  // the Guo source in moment space (the relaxation's forcing term); with CORR it is formed
  // here, before the strain, since half of it joins the non-equilibrium part
  float SF[Q];
  if constexpr (CORR) force_moments(jx, jy, jz, Fx, Fy, Fz, M.inv_rho0, SF);
  const StrainIn<CORR> si = strain_in<CORR>(n, SF);

  float Syu[6], Sch[6];
  float snu = M.s[9];
  float s_strain;  // the s_nu this step's strain is taken with
  if (V.kind == 3) {
    // implicit coupling: the strain at the rate of this very collision
    snu = implicit_rate(P_, drho, jx, jy, jz, si, M, V);
    s_strain = snu;
    if (io.S_out) {
      if (io.emit == 2) {
        float r[Q];
        rates_with(M, snu, r);
        strain_chai_in(P_, drho, jx, jy, jz, r, si, M.inv_rho0, Sch);
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
    s_strain = snu_prev;
    const bool need_yu = io.emit == 1 || (V.kind != 0 && !V.drive_chai);
    const bool need_chai = io.emit == 2 || (V.kind != 0 && V.drive_chai);
    if (need_yu) strain_yu(si.ns, M.s[1], snu_prev, M.inv_rho0, Syu);
    if (need_chai) {
      float r[Q];
      rates_with(M, snu_prev, r);
      strain_chai_in(P_, drho, jx, jy, jz, r, si, M.inv_rho0, Sch);
    }
    if (io.S_out) {
#pragma unroll
      for (int c = 0; c < 6; ++c)
        stream_store(&io.S_out[static_cast<size_t>(c) * G.N + self], io.emit == 2 ? Sch[c] : Syu[c]);
    }
    // viscosity model -> s_nu of this collision (kept for the next step's strain)
    if (V.kind != 0) {
      snu = viscous_rate(V.drive_chai ? strain_sq(Sch) : strain_sq(Syu), V);
      io.snu[self] = snu;
    }
  }

  // Relaxation in moment space, dm_k = -s_k (m_k - m_k^eq) + (1 - s_k/2) S_F,k, taken
  // directly as w_k = dm_k / D_k for the back-transform g += T^T w: the row norms are folded
  // into the rates (M.sd, M.fd; per node for the s_nu rows).
  float w[Q];
  w[0] = 0.0f;
  constexpr float iD3 = 1.0f / static_cast<float>(DV.D[3]);
  w[3] = Fx * iD3;
  w[5] = Fy * iD3;
  w[7] = Fz * iD3;
  static_for<Q>([&](auto ki) {
    constexpr int k = ki;
    if constexpr (k != 0 && k != 3 && k != 5 && k != 7) {
      constexpr float iD = 1.0f / static_cast<float>(DV.D[k]);
      const float c = is_nu_slot(k) ? -snu * iD : M.sd[k];
      w[k] = c * n.m[k];
    }
  });
  if (Fo.mode) {
    if constexpr (!CORR) force_moments(jx, jy, jz, Fx, Fy, Fz, M.inv_rho0, SF);
    static_for<Q>([&](auto ki) {
      constexpr int k = ki;
      if constexpr (k != 0 && k != 3 && k != 5 && k != 7 && k < 16) {
        constexpr float iD = 1.0f / static_cast<float>(DV.D[k]);
        const float c = is_nu_slot(k) ? __builtin_fmaf(-0.5f * iD, snu, iD) : M.fd[k];
        w[k] = __builtin_fmaf(c, SF[k], w[k]);
      }
    });
  }
  if constexpr (PACK) add_scaled_back_transform_packed(w, hp, g);
  else add_scaled_back_transform(w, g);

  if (io.save) {
    // what the adjoint of this step needs: j, and for a strain-dependent viscosity the
    // moments the strain took (Eq. LuoS rows; force-corrected when it is) and its rate
    const size_t N = G.N;
    stream_store(&io.save[self], jx);
    stream_store(&io.save[N + self], jy);
    stream_store(&io.save[2 * N + self], jz);
    if (V.kind != 0) {
      stream_store(&io.save[3 * N + self], si.ns.m[1]);
      stream_store(&io.save[4 * N + self], si.ns.m[9]);
      stream_store(&io.save[5 * N + self], si.ns.m[11]);
      stream_store(&io.save[6 * N + self], si.ns.m[13]);
      stream_store(&io.save[7 * N + self], si.ns.m[14]);
      stream_store(&io.save[8 * N + self], si.ns.m[15]);
      stream_store(&io.save[9 * N + self], s_strain);
    }
  }
}

// ------------------------------------------------------------------------------------------
// The fused step: one thread per node
// ------------------------------------------------------------------------------------------
// XMODE: how a block pulls along x (pull_mode: 0 part rows, 1 whole rows, 2 whole rows with
// the LDS exchange). CORR: the force-corrected strain (a separate instance, so that the plain
// step keeps its register budget).
// FP16 storage without the LDS exchange (whose x-shifted values arrive through LDS as FP32)
// keeps the pulled values packed; that instance fits 80 VGPRs without spilling and is asked
// for 6 waves per SIMD (the 16-bit step moves half the bytes per wave, so it needs the extra
// wave in flight: 4 instead of 5 waves cost it 6.5 %, 6 instead of 5 gained 3.7 %).
template <typename S, int XMODE>
constexpr bool kPackHalves = Codec<S>::kMixedFma && XMODE != 2;
template <typename S, int XMODE, bool CORR>
constexpr int kMinWavesPerEU = (kPackHalves<S, XMODE> && !CORR) ? 6 : 1;

template <typename S, bool WALLS, int XMODE, bool CORR>
__global__ __launch_bounds__(kMaxBlock, (kMinWavesPerEU<S, XMODE, CORR>)) void step_kernel(Geo G, ModelF M, ViscF V,
                                                                                       ForceF Fo, StepIO io) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= G.nx || y >= G.ny) return;
  const Rows<Q, S> r = rows_of<Q, S>(G, x, y, z);
  float g[Q];
  if constexpr (XMODE == 2) pull_rows_staged<Lat, S, WALLS>(static_cast<const S*>(io.src), G, r, y, g);
  else pull_rows<Lat, S, WALLS, XMODE == 1>(static_cast<const S*>(io.src), G, r, y, g);
  node_update<CORR, kPackHalves<S, XMODE>>(g, node_index(G, x, y, z), G, M, V, Fo, io);
  store_rows<Q>(static_cast<S*>(io.dst), G, r, g);
}

template <typename S, bool CORR>
static void launch_step_c(bool walls, const Launch& L, hipStream_t st, const Geo& G, const ModelF& M, const ViscF& V,
                          const ForceF& Fo, const StepIO& io) {
  const int mode = pull_mode(G, L.block);
  // FP32: 4 blocks per CU instead of the 5 its registers allow, in the two shapes where that
  // was measured faster (whole 256-node rows: +2.2-3.0 % at 256^3; 128 x 2 part rows: +1.8 % at
  // 384^3); whole 128-node rows (the 128 x 128 x 512 channel) ran as fast uncapped and 4.4 %
  // slower capped, so other shapes keep their occupancy. The 16-bit steps want more waves,
  // not fewer.
  size_t lds = 0;
  if constexpr (sizeof(S) == 4) {
    if (mode == 2 && L.block.x == 256 && L.block.y == 1) lds = lds_cap_bytes(4, staged_lds_bytes<Lat>());
    else if (mode == 0 && L.block.x == 128 && L.block.y == 2) lds = lds_cap_bytes(4, 0);
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
  Launch L = node_launch(G);
  // 16-bit storage: part-row blocks hold one row segment (128 x 1 ran 1 % faster than 128 x 2
  // in FP16 and BF16 at 384^3, while FP32 runs 3 % faster with two rows)
  if (storage != 0 && pull_mode(G, L.block) == 0 && L.block.y > 1) {
    L.block.y = 1;
    L.grid.y = G.ny;
  }
  switch (storage) {
    case 0: launch_step_t<float>(G.walls != 0, L, st, G, M, V, Fo, io); break;
    case 1: launch_step_t<_Float16>(G.walls != 0, L, st, G, M, V, Fo, io); break;
    case 2: launch_step_t<__bf16>(G.walls != 0, L, st, G, M, V, Fo, io); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace d3q19
}  // namespace lbm
