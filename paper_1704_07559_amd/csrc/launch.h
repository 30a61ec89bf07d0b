// Host-side launchers of the kernels (one translation unit per lattice), called by the C
// ABI, and the sizes of the reductions. Nothing here changes the code of the step kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace lbm {

// Reductions: 8 doubles per block (at most kReduceBlocks blocks, each taking whole x-rows),
// then one block folds the partials in a fixed order.
constexpr int kReduceBlocks = 4096;
constexpr int kReduceVals = 8;

namespace d3q19 {
hipError_t launch_init(int storage, const Geo&, const ModelF&, void* buf, float* snu, const float* rho_u,
                       const float* grad_u, hipStream_t);
hipError_t launch_step(int storage, const Geo&, const ModelF&, const ViscF&, const ForceF&, const StepIO&,
                       hipStream_t);
hipError_t launch_strain(int storage, const Geo&, const ModelF&, const ViscF&, const ForceF&, const void* buf,
                         const float* snu, int kind, float* S_out, hipStream_t);
hipError_t launch_get(int storage, const Geo&, const void* buf, float* canon, hipStream_t);
hipError_t launch_set(int storage, const Geo&, void* buf, const float* canon, hipStream_t);
hipError_t launch_reduce(int storage, const Geo&, const ModelF&, const ViscF&, const ForceF&, const void* buf,
                         const float* snu, double* partials, double* out, hipStream_t);
// in_rows / out_rows: planes 0..18 of lam_in / lam_out row-interleaved (as the population
// buffers) instead of canonical planes; a multi-step sweep keeps its intermediate states so.
hipError_t launch_adjoint_step(const Geo&, const ModelF&, const ViscF&, const ForceF&, const float* rec,
                               const float* lam_in, float* lam_out, float* grad_force, hipStream_t,
                               bool in_rows = false, bool out_rows = false);
hipError_t launch_loss_seed(int storage, const Geo&, const ModelF&, const ViscF&, const ForceF&, const void* buf,
                            const float* snu, float* lam_out, float* grad_force, double* partials, double* out,
                            hipStream_t);
hipError_t launch_init_adjoint(const Geo&, const ModelF&, const float* rho_u, const float* lam0, float* grad_u0,
                               hipStream_t);
}  // namespace d3q19

namespace d2q9 {
hipError_t launch_init(int storage, const Geo&, const ModelF&, void* buf, float* snu, const float* rho_u,
                       const float* grad_u, hipStream_t);
hipError_t launch_step(int storage, const Geo&, const ModelF&, const ViscF&, const ForceF&, const StepIO&,
                       hipStream_t);
hipError_t launch_strain(int storage, const Geo&, const ModelF&, const ViscF&, const ForceF&, const void* buf,
                         const float* snu, int kind, float* S_out, hipStream_t);
hipError_t launch_get(int storage, const Geo&, const void* buf, float* canon, hipStream_t);
hipError_t launch_set(int storage, const Geo&, void* buf, const float* canon, hipStream_t);
hipError_t launch_reduce(int storage, const Geo&, const ModelF&, const ViscF&, const ForceF&, const void* buf,
                         const float* snu, double* partials, double* out, hipStream_t);
// Two steps in one launch (boxes at least 256 wide, periodic or with walls in y): src -> dst, the lagged s_nu field (if any) snu_in -> snu_out (distinct buffers);
// S_out (or nullptr) receives the strain (emit 1 Yu, 2 Chai) of the second step. The result
// equals two launch_step calls bit for bit.
bool pair_supported(const Geo&);
hipError_t launch_pair(int storage, const Geo&, const ModelF&, const ViscF&, const ForceF&, const void* src, void* dst,
                       const float* snu_in, float* snu_out, float* S_out, int emit, hipStream_t);
}  // namespace d2q9

namespace d3q15 {
hipError_t launch_init(int storage, const Geo&, const ModelF&, void* buf, float* snu, const float* rho_u,
                       const float* grad_u, hipStream_t);
hipError_t launch_step(int storage, const Geo&, const ModelF&, const ViscF&, const ForceF&, const StepIO&,
                       hipStream_t);
hipError_t launch_strain(int storage, const Geo&, const ModelF&, const ViscF&, const ForceF&, const void* buf,
                         const float* snu, int kind, float* S_out, hipStream_t);
hipError_t launch_get(int storage, const Geo&, const void* buf, float* canon, hipStream_t);
hipError_t launch_set(int storage, const Geo&, void* buf, const float* canon, hipStream_t);
hipError_t launch_reduce(int storage, const Geo&, const ModelF&, const ViscF&, const ForceF&, const void* buf,
                         const float* snu, double* partials, double* out, hipStream_t);
}  // namespace d3q15

// Fixed device scratch of the allocation-free adjoint sweep: room for one adjoint state of up
// to 64 MiB (A planes of N floats), held by every device the library runs on.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;

// Address of that scratch on the device of `stream` (looked up on the first call per device;
// no allocation).
hipError_t noalloc_scratch(hipStream_t stream, void** out);

// Fold nblocks partials into out[0..7]. rho0 > 0 (the diagnostics): slot 6 arrives as the
// largest |j|^2 and leaves as max |u| = sqrt(.) / rho0.
hipError_t launch_reduce_final(const double* partials, int nblocks, double* out, hipStream_t, double rho0 = 0.0);
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t);

}  // namespace lbm
