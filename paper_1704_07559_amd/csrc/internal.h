// Internal declarations shared by the kernels and the C ABI layer (not installed).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "codec.h"
#include "static_for.h"

namespace lbm {

// Grid geometry. Fields are SoA with x fastest: element (c, z, y, x) at c*N + (z*ny+y)*nx + x.
struct Geo {
  int nx, ny, nz;
  unsigned N;  // nx*ny*nz (< 2^31 elements per component)
  int walls;   // halfway bounce-back at y = -1/2 and y = ny - 1/2
};

// Row norms D_k = sum_i T_ki^2 of the D3Q19 transformation matrix (checked against T where
// the device code derives them).
constexpr int kD3Q19RowNorm[19] = {19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8};

// Model constants in FP32. For D3Q19, sd and fd fold the row norms into the relaxation:
// sd[k] = -s_k / D_k and fd[k] = (1 - s_k / 2) / D_k (zero for the other lattices).
struct ModelF {
  float rho0, inv_rho0;
  float s[19];
  float om_eps, om_epsj, om_xx;
  float sd[19], fd[19];
};

struct ViscF {
  int kind;        // 0 const, 1 Smagorinsky (lagged), 2 power law (lagged), 3 Smagorinsky (implicit)
  int drive_chai;  // 1: the Chai strain drives the viscosity, 0: the Yu strain
  float nu0, csmag2, Kpl, npl, numin, numax;
};

struct ForceF {
  int mode;  // 0 none, 1 uniform, 2 field
  float F[3];
  const float* field;
  int strain_corr;  // strains take the non-equilibrium part plus half the Guo source (mode != 0 only)
};

// Node coordinates of the three source positions along each axis, indexed by c + 1:
// a pull reads element i at x - c_i, so c = -1 -> x + 1, c = 0 -> x, c = +1 -> x - 1.
// Offsets are in elements of one plane of a node-indexed array; `self` is the node itself.
struct Nbr {
  unsigned xs[3], ys[3], zs[3];
  unsigned self;
};

__device__ __forceinline__ Nbr neighbours(const Geo& G, int x, int y, int z) {
  Nbr n;
  const unsigned nx = G.nx, nxy = static_cast<unsigned>(G.nx) * G.ny;
  n.xs[0] = (x == G.nx - 1) ? 0u : x + 1;
  n.xs[1] = x;
  n.xs[2] = (x == 0) ? nx - 1 : x - 1;
  n.ys[0] = ((y == G.ny - 1) ? 0u : y + 1) * nx;
  n.ys[1] = y * nx;
  n.ys[2] = ((y == 0) ? G.ny - 1u : y - 1) * nx;
  n.zs[0] = ((z == G.nz - 1) ? 0u : z + 1) * nxy;
  n.zs[1] = z * nxy;
  n.zs[2] = ((z == 0) ? G.nz - 1u : z - 1) * nxy;
  n.self = n.zs[1] + n.ys[1] + x;
  return n;
}

// The same offsets in bytes for elements of type S (N < 2^30 nodes keeps every byte offset
// inside one plane below 2^32).
template <typename S>
__device__ __forceinline__ Nbr in_bytes(const Nbr& n) {
  constexpr unsigned b = sizeof(S);
  Nbr r;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r.xs[k] = n.xs[k] * b;
    r.ys[k] = n.ys[k] * b;
    r.zs[k] = n.zs[k] * b;
  }
  r.self = n.self * b;
  return r;
}

// Load/store at a wave-uniform base plus a 32-bit byte offset (the SGPR-base + VGPR-offset
// addressing form of global memory instructions).
template <typename S>
__device__ __forceinline__ float load_at(const void* base, unsigned byte_off) {
  return Codec<S>::load(reinterpret_cast<const S*>(static_cast<const char*>(base) + byte_off));
}
template <typename S>
__device__ __forceinline__ float load_at_cached(const void* base, unsigned byte_off) {
  return Codec<S>::load_cached(reinterpret_cast<const S*>(static_cast<const char*>(base) + byte_off));
}
template <typename S>
__device__ __forceinline__ void store_at(void* base, unsigned byte_off, float v) {
  Codec<S>::store(reinterpret_cast<S*>(static_cast<char*>(base) + byte_off), v);
}

// True when population i arriving at row y crossed a y-wall (its source row y - c_y is
// outside 0..ny-1); bounce-back then takes the opposite population of the same node.
template <int CYI>
__device__ __forceinline__ bool crosses_wall(const Geo& G, int y) {
  if constexpr (CYI == 0) return false;
  else if constexpr (CYI > 0) return G.walls && y == 0;
  else return G.walls && y == G.ny - 1;
}

// Pull along -c on a node-indexed array (structure of arrays, plane i at i * N): element i
// of node x - c_i (periodic), or element opp(i) of x across a y-wall. Used for the adjoint
// state, whose transposed streaming is a pull along -c; nb holds byte offsets for S.
template <class L, typename S, bool WALLS = true>
__device__ __forceinline__ void pull(const S* __restrict__ src, const Geo& G, const Nbr& nb, int y, float (&g)[L::Q]) {
  const char* cb = reinterpret_cast<const char*>(src);
  const size_t plane = static_cast<size_t>(G.N) * sizeof(S);
  static_for<L::Q>([&](auto ii) {
    constexpr int i = ii;
    const unsigned off = nb.zs[L::cz(i) + 1] + nb.ys[L::cy(i) + 1] + nb.xs[L::cx(i) + 1];
    if constexpr (WALLS && L::cy(i) != 0) {
      if (crosses_wall<L::cy(i)>(G, y)) {
        g[i] = load_at<S>(cb + L::opp(i) * plane, nb.self);
        return;
      }
    }
    g[i] = load_at<S>(cb + i * plane, off);
  });
}

// ---- internal population buffers -------------------------------------------------------
// The two state buffers are row-interleaved: element (i, z, y, x) sits at
// ((z * ny + y) * Q + i) * nx + x, so the Q populations of one x-row are Q consecutive runs
// of nx elements. A wave's 2 Q streams then fall into the few DRAM pages of the 3 x 3 rows
// around it instead of Q planes N elements apart. Addresses are a wave-uniform 64-bit base
// (buffer + z-plane + population run) plus a 32-bit per-lane byte offset within the z-plane
// (ny * Q * nx * sizeof(S) < 2^32, checked by lbm_init).
template <int Q, typename S>
struct Rows {
  size_t zb[3];    // byte offsets of the z-planes z + 1, z, z - 1 (indexed by c + 1)
  unsigned yb[3];  // byte offsets of the rows y + 1, y, y - 1 within a z-plane
  unsigned xb[3];  // byte offsets of x + 1, x, x - 1 within a population run
  unsigned self;   // yb[1] + xb[1]
};

template <int Q, typename S>
__device__ __forceinline__ Rows<Q, S> rows_of(const Geo& G, int x, int y, int z) {
  Rows<Q, S> r;
  constexpr unsigned b = sizeof(S);
  const unsigned row = static_cast<unsigned>(Q) * G.nx * b;
  const size_t plane = static_cast<size_t>(G.ny) * row;
  r.xb[0] = ((x == G.nx - 1) ? 0u : x + 1) * b;
  r.xb[1] = x * b;
  r.xb[2] = ((x == 0) ? G.nx - 1u : x - 1) * b;
  r.yb[0] = ((y == G.ny - 1) ? 0u : y + 1) * row;
  r.yb[1] = y * row;
  r.yb[2] = ((y == 0) ? G.ny - 1u : y - 1) * row;
  r.zb[0] = ((z == G.nz - 1) ? 0u : z + 1) * plane;
  r.zb[1] = z * plane;
  r.zb[2] = ((z == 0) ? G.nz - 1u : z - 1) * plane;
  r.self = r.yb[1] + r.xb[1];
  return r;
}

// Pull streaming (the left side of Eq. mrteq) from an internal buffer: canonical g_i(x, n)
// is the post-collision population i of node x - c_i (periodic), or of population opp(i)
// at x across a wall. With WALLS false the bounce test is compiled out.
// Cache policy: every population is read once per step, so loads are nontemporal, except
// (ROW_BLOCKS false) the x-shifted populations when a block holds only part of an x-row:
// their first or last cache line is also read by the neighbouring block, which may run on
// another XCD, and a streaming hint there costs a refetch from HBM.
template <class L, typename S, bool WALLS = true, bool ROW_BLOCKS = true>
__device__ __forceinline__ void pull_rows(const S* __restrict__ src, const Geo& G, const Rows<L::Q, S>& r, int y,
                                          float (&g)[L::Q]) {
  const char* cb = reinterpret_cast<const char*>(src);
  const size_t run = static_cast<size_t>(G.nx) * sizeof(S);
  static_for<L::Q>([&](auto ii) {
    constexpr int i = ii;
    if constexpr (WALLS && L::cy(i) != 0) {
      if (crosses_wall<L::cy(i)>(G, y)) {
        g[i] = load_at<S>(cb + r.zb[1] + L::opp(i) * run, r.self);
        return;
      }
    }
    const char* base = cb + r.zb[L::cz(i) + 1] + i * run;
    const unsigned off = r.yb[L::cy(i) + 1] + r.xb[L::cx(i) + 1];
    if constexpr (L::cx(i) != 0 && !ROW_BLOCKS) g[i] = load_at_cached<S>(base, off);
    else g[i] = load_at<S>(base, off);
  });
}

// The populations with c_x != 0 (the x-shifted ones) of a lattice: their number and the
// LDS slot of each.
template <class L>
struct XShifted {
  static constexpr int count() {
    int n = 0;
    for (int i = 0; i < L::Q; ++i) n += L::cx(i) != 0;
    return n;
  }
  static constexpr int N = count();
  static constexpr int slot(int i) {
    int n = 0;
    for (int k = 0; k < i; ++k) n += L::cx(k) != 0;
    return n;
  }
};

// Pull with the x-shifted populations exchanged through LDS, for blocks of whole rows:
// blockDim.x == nx >= 64 (so at most 4 rows per 256-thread block) and every thread of the
// block inside the box. Each thread loads its own aligned element of each x-shifted source
// row into LDS; after one barrier it takes its neighbour's element (periodic within the row)
// from there. Every global load is then aligned to the wave's segment, instead of the
// x-shifted loads each touching one more cache line than they use. All threads of the block
// must call it.
template <class L, typename S, bool WALLS>
__device__ __forceinline__ void pull_rows_staged(const S* __restrict__ src, const Geo& G, const Rows<L::Q, S>& r,
                                                 int y, float (&g)[L::Q]) {
  using X = XShifted<L>;
  __shared__ float sh[X::N][256];
  const char* cb = reinterpret_cast<const char*>(src);
  const size_t run = static_cast<size_t>(G.nx) * sizeof(S);
  const unsigned row = threadIdx.y * blockDim.x;
  static_for<L::Q>([&](auto ii) {
    constexpr int i = ii;
    const char* base = cb + r.zb[L::cz(i) + 1] + i * run;
    const unsigned off = r.yb[L::cy(i) + 1] + r.xb[1];
    if constexpr (L::cx(i) != 0) {
      sh[X::slot(i)][row + threadIdx.x] = load_at<S>(base, off);
    } else {
      if constexpr (WALLS && L::cy(i) != 0) {
        if (crosses_wall<L::cy(i)>(G, y)) {
          g[i] = load_at<S>(cb + r.zb[1] + L::opp(i) * run, r.self);
          return;
        }
      }
      g[i] = load_at<S>(base, off);
    }
  });
  __syncthreads();
  static_for<L::Q>([&](auto ii) {
    constexpr int i = ii;
    if constexpr (L::cx(i) != 0) {
      if constexpr (WALLS && L::cy(i) != 0) {
        if (crosses_wall<L::cy(i)>(G, y)) {
          g[i] = load_at<S>(cb + r.zb[1] + L::opp(i) * run, r.self);
          return;
        }
      }
      g[i] = sh[X::slot(i)][row + r.xb[L::cx(i) + 1] / sizeof(S)];
    }
  });
}

// The structure-of-arrays counterpart of pull_rows_staged for node-indexed arrays (the
// adjoint state): whole-row blocks, the x-shifted elements exchanged through LDS. All
// threads of the block must call it.
template <class L, typename S, bool WALLS>
__device__ __forceinline__ void pull_staged(const S* __restrict__ src, const Geo& G, const Nbr& nb, int y,
                                            float (&g)[L::Q]) {
  using X = XShifted<L>;
  __shared__ float sh[X::N][256];
  const char* cb = reinterpret_cast<const char*>(src);
  const size_t plane = static_cast<size_t>(G.N) * sizeof(S);
  const unsigned row = threadIdx.y * blockDim.x;
  static_for<L::Q>([&](auto ii) {
    constexpr int i = ii;
    const unsigned off = nb.zs[L::cz(i) + 1] + nb.ys[L::cy(i) + 1] + nb.xs[1];
    if constexpr (L::cx(i) != 0) {
      sh[X::slot(i)][row + threadIdx.x] = load_at<S>(cb + i * plane, off);
    } else {
      if constexpr (WALLS && L::cy(i) != 0) {
        if (crosses_wall<L::cy(i)>(G, y)) {
          g[i] = load_at<S>(cb + L::opp(i) * plane, nb.self);
          return;
        }
      }
      g[i] = load_at<S>(cb + i * plane, off);
    }
  });
  __syncthreads();
  static_for<L::Q>([&](auto ii) {
    constexpr int i = ii;
    if constexpr (L::cx(i) != 0) {
      if constexpr (WALLS && L::cy(i) != 0) {
        if (crosses_wall<L::cy(i)>(G, y)) {
          g[i] = load_at<S>(cb + L::opp(i) * plane, nb.self);
          return;
        }
      }
      g[i] = sh[X::slot(i)][row + nb.xs[L::cx(i) + 1] / sizeof(S)];
    }
  });
}

// How a step launch pulls along x: 0 blocks hold part of a row (x-shifted loads cached, as
// a neighbouring block reads their edge lines too); 1 blocks hold whole rows with masked
// lanes (every load streams); 2 blocks hold whole rows exactly (LDS exchange above).
inline int pull_mode(const Geo& G, const dim3& block) {
  const int bx = static_cast<int>(block.x);
  if (bx == G.nx && bx >= 64 && G.ny % static_cast<int>(block.y) == 0) return 2;
  return bx >= G.nx ? 1 : 0;
}

// Inverse of pull_rows: write canonical g_i(x) to the internal slot it is pulled from.
template <class L, typename S>
__device__ __forceinline__ void scatter_rows(S* __restrict__ dst, const Geo& G, const Rows<L::Q, S>& r, int y,
                                             const float (&g)[L::Q]) {
  char* cb = reinterpret_cast<char*>(dst);
  const size_t run = static_cast<size_t>(G.nx) * sizeof(S);
  static_for<L::Q>([&](auto ii) {
    constexpr int i = ii;
    if (crosses_wall<L::cy(i)>(G, y)) {
      store_at<S>(cb + r.zb[1] + L::opp(i) * run, r.self, g[i]);
    } else {
      store_at<S>(cb + r.zb[L::cz(i) + 1] + i * run, r.yb[L::cy(i) + 1] + r.xb[L::cx(i) + 1], g[i]);
    }
  });
}

// Store post-collision populations at the node itself (aligned, coalesced).
template <int Q, typename S>
__device__ __forceinline__ void store_rows(S* __restrict__ dst, const Geo& G, const Rows<Q, S>& r,
                                           const float (&g)[Q]) {
  char* cb = reinterpret_cast<char*>(dst) + r.zb[1];
  const size_t run = static_cast<size_t>(G.nx) * sizeof(S);
  if constexpr (sizeof(S) == 2) {
    // 16-bit storage: one packed conversion rounds two populations (low and high half of
    // one register, each stored from its half), and the lane offset is re-materialised next
    // to the stores (the empty asm emits nothing) so that they take the scalar-base form
    // instead of a 64-bit vector add each; 29 fewer VALU instructions per node. (For FP32
    // storage the same addressing measured 1 % slower at 256^3, so FP32 keeps the plain form.)
    unsigned self = r.self;
    asm volatile("" : "+v"(self));
    static_for<Q / 2>([&](auto pp) {
      constexpr int i = 2 * pp;
      const unsigned w = Codec<S>::encode2(g[i], g[i + 1]);
      stream_store(reinterpret_cast<unsigned short*>(cb + i * run + self), static_cast<unsigned short>(w & 0xffffu));
      stream_store(reinterpret_cast<unsigned short*>(cb + (i + 1) * run + self), static_cast<unsigned short>(w >> 16));
    });
    if constexpr (Q % 2 != 0) {
      // the odd population alone: its FP32 value is rounded to 16 bits as it is. (An FMA
      // producing it from FP16 operands would otherwise be fused with the rounding into one
      // v_fma_mixlo_f16, rounding the exact result once instead of the FP32 result.)
      float last = g[Q - 1];
      if constexpr (Codec<S>::kMixedFma) asm("" : "+v"(last));
      store_at<S>(cb + (Q - 1) * run, self, last);
    }
  } else {
    static_for<Q>([&](auto ii) {
      constexpr int i = ii;
      store_at<S>(cb + i * run, r.self, g[i]);
    });
  }
}

// Node index of (x, y, z) in the node-indexed fields (s_nu, forces, strain, canonical
// populations, adjoint states): (z * ny + y) * nx + x.
__device__ __forceinline__ unsigned node_index(const Geo& G, int x, int y, int z) {
  return (static_cast<unsigned>(z) * G.ny + y) * G.nx + x;
}

// A node's index in the node-indexed fields together with its internal-buffer addresses.
template <int Q, typename S>
struct Node {
  unsigned self;
  Rows<Q, S> rows;
};

template <int Q, typename S>
__device__ __forceinline__ Node<Q, S> node_at(const Geo& G, int x, int y, int z) {
  return Node<Q, S>{node_index(G, x, y, z), rows_of<Q, S>(G, x, y, z)};
}

// Store Q values of node `self_bytes` (byte offset for S) into a node-indexed array
// (structure of arrays, plane i at i * N): canonical populations and adjoint states.
template <int Q, typename S>
__device__ __forceinline__ void store_local(S* __restrict__ dst, const Geo& G, unsigned self_bytes,
                                            const float (&g)[Q]) {
  char* cb = reinterpret_cast<char*>(dst);
  const size_t plane = static_cast<size_t>(G.N) * sizeof(S);
  static_for<Q>([&](auto ii) {
    constexpr int i = ii;
    store_at<S>(cb + i * plane, self_bytes, g[i]);
  });
}

// Square root and reciprocal as the single hardware instructions (within 1 ulp; the
// correctly rounded library forms cost about ten instructions each, on every node). Their
// arguments here are never subnormal where it matters: S:S >= 0 (a subnormal |S| changes
// nu by nothing representable) and 3 nu + 1/2 >= 1/2.
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// s_nu = 1 / (3 nu + 1/2) from the strain magnitude |S| = sqrt(2 S:S).
__device__ __forceinline__ float viscous_rate(float SS, const ViscF& V) {
  const float gamma = fast_sqrt(2.0f * SS);
  float nu;
  if (V.kind == 1) {
    nu = V.nu0 + V.csmag2 * gamma;
  } else {
    if (gamma > 0.0f) nu = V.Kpl * powf(gamma, V.npl - 1.0f);
    else nu = (V.npl < 1.0f) ? V.numax : ((V.npl > 1.0f) ? V.numin : V.Kpl);
    nu = fminf(fmaxf(nu, V.numin), V.numax);
  }
  return fast_rcp(3.0f * nu + 0.5f);
}

// d nu / d gamma of the lagged models (zero where the power law is clamped or gamma = 0).
__device__ __forceinline__ float viscous_slope(float gamma, const ViscF& V) {
  if (V.kind == 1) return V.csmag2;
  if (!(gamma > 0.0f)) return 0.0f;
  const float nu = V.Kpl * powf(gamma, V.npl - 1.0f);
  return (nu > V.numin && nu < V.numax) ? (V.npl - 1.0f) * nu / gamma : 0.0f;
}

// Implicit Smagorinsky coupling. Every strain formula here (Yu, Chai, and the Yu-type
// formulas of the other lattices) is affine in s_nu: S(s) = P + s A, P from the rows relaxed
// at the other rates, A from the s_nu rows. Returns the s > 0 solving
//   s (c + k |P + s A|) = 1,  c = 3 nu0 + 1/2, k = 3 C_s^2, |S| = sqrt(2 S:S),
// whose left side increases with s. NC = 6 (3D, xx yy zz xy xz yz) or 3 (2D, xx yy xy);
// off-diagonal components count twice in S:S. Newton from the root of the P = 0 case,
// k sqrt(2 A:A) s^2 + c s - 1 = 0; three steps reach FP32 resolution. Every product that
// meets a sum is an explicit FMA, so that the rate rounds the same in every kernel (left to
// the compiler, which product of a sum of two products gets fused depends on the code around).
template <int NC>
__device__ __forceinline__ float implicit_smagorinsky(const float (&P)[NC], const float (&A)[NC], float nu0,
                                                     float csmag2) {
  static_assert(NC == 6 || NC == 3, "3D or 2D symmetric tensor");
  constexpr int ndiag = NC == 6 ? 3 : 2;
  const float c = __builtin_fmaf(3.0f, nu0, 0.5f), k = 3.0f * csmag2;
  float PP = P[0] * P[0], PA = P[0] * A[0], AA = A[0] * A[0];
#pragma unroll
  for (int i = 1; i < NC; ++i) {
    const float w = i < ndiag ? 1.0f : 2.0f;
    PP = __builtin_fmaf(w * P[i], P[i], PP);
    PA = __builtin_fmaf(w * P[i], A[i], PA);
    AA = __builtin_fmaf(w * A[i], A[i], AA);
  }
  const float q = k * fast_sqrt(2.0f * AA);
  float s = 2.0f * fast_rcp(c + fast_sqrt(__builtin_fmaf(c, c, 4.0f * q)));
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    const float r = fast_sqrt(fmaxf(2.0f * __builtin_fmaf(s, __builtin_fmaf(s, AA, 2.0f * PA), PP), 0.0f));
    const float dr = r > 0.0f ? 2.0f * __builtin_fmaf(s, AA, PA) * fast_rcp(r) : 0.0f;
    const float ckr = __builtin_fmaf(k, r, c);
    const float f = __builtin_fmaf(s, ckr, -1.0f);
    s = __builtin_fmaf(-f, fast_rcp(__builtin_fmaf(s * k, dr, ckr)), s);
  }
  return s;
}

// Launch shape for the node-parallel kernels: one thread per node, blocks of (TX, TY)
// nodes (at most kMaxBlock threads), grid (ceil(nx/TX), ceil(ny/TY), nz).
constexpr int kMaxBlock = 256;

struct Launch {
  dim3 grid, block;
};

inline Launch node_launch(const Geo& G) {
  // 256-thread blocks (one wave per SIMD of a CU). The row segment tx is the widest power
  // of two (<= 256) dividing nx when nx is a multiple of 64; ragged rows use the smallest
  // power of two covering nx (masked lanes).
  int tx = 256;
  if (G.nx % 64 == 0) {
    while (G.nx % tx != 0) tx /= 2;
  } else {
    tx = 1;
    while (tx < G.nx && tx < 256) tx *= 2;
  }
  int ty = 256 / tx;
  int py = 1;
  while (py < G.ny) py *= 2;
  if (ty > py) ty = py;
  Launch L;
  L.block = dim3(tx, ty, 1);
  L.grid = dim3((G.nx + tx - 1) / tx, (G.ny + ty - 1) / ty, G.nz);
  return L;
}

// Occupancy caps. Some of the streaming kernels run faster with fewer blocks per CU than their
// registers allow (fewer address streams in flight at once per CU). A launch caps them by
// reserving LDS the kernel does not use: a 256-thread block holding `total` bytes of LDS lets
// `blocks` of them share a CU (measured on MI355X with blocks that only sleep, 160 KB of LDS
// per CU: 5 blocks of exactly 32 KB do not fit, 4 of 40 KB do; the values below sit inside the
// measured ranges). Returns the dynamic LDS to request on top of the kernel's static LDS
// (0: no cap). Results do not change: the reserved LDS is never touched.
inline size_t lds_cap_bytes(int blocks, size_t static_lds) {
  size_t total = 0;
  switch (blocks) {
    case 3: total = 47104; break;
    case 4: total = 36864; break;
    case 5: total = 28672; break;
    case 6: total = 23552; break;
    default: return 0;
  }
  return total > static_lds ? total - static_lds : 0;
}

// LDS of the exchange of x-shifted values (pull_rows_staged, pull_staged) for a lattice.
template <class L>
constexpr size_t staged_lds_bytes() {
  return static_cast<size_t>(XShifted<L>::N) * 256 * sizeof(float);
}

// Launch arguments of one step.
struct StepIO {
  const void* src;
  void* dst;
  float* snu;     // lagged s_nu field (variable viscosity) or nullptr
  float* S_out;   // strain output or nullptr
  int emit;       // 1 Yu, 2 Chai
  float* save;    // per-step adjoint record (save_planes(V) * N floats) or nullptr
};

// Planes of the per-step record the step writes for the adjoint: j (3), plus, for a
// strain-dependent viscosity, m^neq of rows 1, 9, 11, 13, 14, 15 and the strain's s_nu.
inline int save_planes(const ViscF& V) { return V.kind == 0 ? 3 : 10; }

}  // namespace lbm
