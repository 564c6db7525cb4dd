// Host launchers of the gfx950 kernels (kernels.hip).  All are asynchronous
// on `st` and return the launch status.
#pragma once
#include <hip/hip_runtime.h>

#include "ctx.h"

namespace ckks {

// Forward NTT of rows [0, rows) of src into dst (may alias), skipping [skip_lo, skip_hi).
hipError_t launch_ntt(const Ctx& c, const uint32_t* src, uint32_t* dst, int rows, RowMap rm,
                      int skip_lo, int skip_hi, hipStream_t st);
// Inverse NTT; each row is scaled by scale[pidx - scale_off] (or N^-1 if scale is null).
hipError_t launch_intt(const Ctx& c, const uint32_t* src, uint32_t* dst, int rows, RowMap rm,
                       int skip_lo, int skip_hi, const uint2* scale, int scale_off,
                       hipStream_t st);
// z_r = sum_{i < nin} y_i * Tt[r * tstride + i] mod prime(r), rows [0, nrows) minus the skip range.
hipError_t launch_bconv(const Ctx& c, RowMap rm, const uint32_t* y, int nin, uint32_t* out,
                        int nrows, int skip_lo, int skip_hi, const uint32_t* Tt, int tstride,
                        hipStream_t st);
hipError_t launch_inner_product(const Ctx& c, RowMap rm, const uint32_t* M, int beta, int nrows,
                                const uint32_t* evk, uint32_t* acc, hipStream_t st);
hipError_t launch_tensor(const Ctx& c, const uint32_t* ct1, const uint32_t* ct2, int L,
                         uint32_t* out, hipStream_t st);
hipError_t launch_automorph(const Ctx& c, const uint32_t* in, uint32_t* out, int rows, uint32_t g,
                            hipStream_t st);
hipError_t launch_moddown_combine(const Ctx& c, int L, const uint32_t* acc, const uint32_t* z,
                                  const uint32_t* add, uint32_t* out, hipStream_t st);
hipError_t launch_add(const Ctx& c, int rows, const uint32_t* a, const uint32_t* b, uint32_t* out,
                      hipStream_t st);
hipError_t launch_broadcast_mod(const Ctx& c, int rows, const uint32_t* t, uint32_t* bc,
                                hipStream_t st);
hipError_t launch_sub_scale(const Ctx& c, int rows, const uint32_t* a, const uint32_t* v,
                            const uint2* qinv, uint32_t* out, hipStream_t st);

hipError_t launch_pmult_sum(const Ctx& c, const uint32_t* const* cts, const uint32_t* const* pts, int nb,
                            int L, uint32_t* out, hipStream_t st);
hipError_t launch_pmult_sums(const Ctx& c, const uint32_t* const* cts, int nb, const uint32_t* const* pts,
                             int ng, int L, uint32_t* const* outs, hipStream_t st);
hipError_t launch_ct_add(const Ctx& c, const uint32_t* a, const uint32_t* b, int L, uint32_t* out,
                         hipStream_t st);

}  // namespace ckks
