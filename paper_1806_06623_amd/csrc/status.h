// Status record of the last solve enqueued on a workspace (it occupies the
// first SPP_STATUS_BYTES of every workspace; the fields follow), and the gate
// through which a kernel sequence runs conditionally on the device.
//
// The first kernel of a solve clears the record.  The inverse FFT sets
// `nonfinite` when it stores a value of Phi that is not finite (a NaN or an
// infinity in rho, or an overflow, reaches Phi through every stage).  The
// mixed form's residual kernels record max |r_k| of each residual and the
// gate kernel decides whether the refinement contracted; its FP64 fallback
// solve runs only when `fallback` is set.  spp_solve_status reads the record
// after the stream has finished.
#pragma once
#include <cstddef>

struct alignas(256) spp_status_record {
    unsigned nonfinite;           // Phi holds a non-finite value
    unsigned fallback;            // gate of the FP64 fallback solve of the mixed form (1: run it)
    unsigned not_contracted;      // a refinement step of the mixed form did not contract
    unsigned refine_iters;        // refinement steps the mixed form took
    unsigned long long rmax[20];  // max |r_k| of residual k (k = 0: the source), as IEEE-754 bits
};

constexpr size_t SPP_STATUS_BYTES = 256;
static_assert(sizeof(spp_status_record) == SPP_STATUS_BYTES, "status record");
constexpr int SPP_MAX_REFINE = 16;

// A kernel launched with a gate returns at once unless the gate word is
// non-zero; launched with NULL it always runs.
__device__ __forceinline__ bool spp_gate_closed(const unsigned* gate) { return gate != nullptr && *gate == 0u; }

// Zero the status record (first kernel of a solve, by the first workgroup of
// the solve).
__device__ __forceinline__ void spp_status_clear(spp_status_record* rec, bool first_block)
{
    if (rec && first_block && threadIdx.x < SPP_STATUS_BYTES / 8)
        reinterpret_cast<unsigned long long*>(rec)[threadIdx.x] = 0ull;
}

// Several right-hand sides of one grid in one launch (batched solves): RHS r
// reads rho[r], writes phi[r], scales by scale[r] and owns the spectral field
// at r * xstride doubles and the status record at r (its workgroups are
// consecutive).  With rho == nullptr (forward) / phi == nullptr (inverse) the
// launch is a single solve.
struct spp_batch_view {
    const double* const* rho = nullptr;
    double* const* phi = nullptr;
    const double* scale = nullptr;
    size_t xstride = 0;
};
