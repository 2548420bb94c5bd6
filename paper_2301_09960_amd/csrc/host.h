// Host-side helpers shared by the single-product and batched C-ABI code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mp {
namespace host {

constexpr int kNumFmtH = 4;
extern const int kCompsH[kNumFmtH];

// Options of the calling host thread.
int thread_mode(int fmt);
int layout_for(int fmt);
// The INT8 tile configuration this thread forces (0: chosen by size).
int int8_tile_override();
int split_kernel_override();
int last_slice_option();
int slices_for(int fmt, int mode, int64_t k);
void set_last_slices(int D);

// The shift ceil((S + log2 k) / 2) of Algorithm 1.
int rho_of(int S, int64_t k);

// BLAS-style argument check of one product (0, -position, or MPGEMM_ERR_TOO_LARGE).
int validate(int m, int n, int k, const void *A, int lda, const void *B, int ldb, const void *C, int ldc);

// 0 if the current device is a gfx950, else an MPGEMM_ERR_* code.
int check_device_cached();

int hip_status(hipError_t e);

// Stage-timing hooks (mpgemm_profile_*): events before/after a unit of work.
bool profiling();
void profile_mark3(hipEvent_t (&ev)[3]);
void profile_commit(hipEvent_t (&ev)[3]);

}  // namespace host
}  // namespace mp
