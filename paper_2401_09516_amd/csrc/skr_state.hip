// Copies of the carried recycle space between the context's workspace and caller buffers
// (checkpoint and resume of a chain: skr_recycle_get / skr_recycle_set).
#include "skr_internal.hpp"

namespace skr {

// Copy of an n x k column block between the caller's FP64 layout (leading dimension ldc) and the
// workspace U (leading dimension ldu, element type BT): to_u rounds to BT (FP32: to nearest even),
// otherwise widens exactly. Grid: (row blocks, k).
template <typename BT>
__global__ __launch_bounds__(ROWS) void k_copy_u(double* __restrict__ c, long ldc, BT* __restrict__ u, long ldu,
                                                 int n, int to_u) {
    const int i = blockIdx.x * ROWS + threadIdx.x;
    const long j = blockIdx.y;
    if (i >= n) return;
    if (to_u) u[j * ldu + i] = (BT)c[j * ldc + i];
    else c[j * ldc + i] = (double)u[j * ldu + i];
}

void launch_copy_u(hipStream_t s, const Work& w, double* c, long ldc, int kcols, int to_u) {
    if (kcols <= 0 || w.n <= 0) return;
    const dim3 grid((w.n + ROWS - 1) / ROWS, kcols);
    if (w.mixed)
        hipLaunchKernelGGL(k_copy_u<float>, grid, dim3(ROWS), 0, s, c, ldc, reinterpret_cast<float*>(w.U),
                           (long)w.ld, w.n, to_u);
    else
        hipLaunchKernelGGL(k_copy_u<double>, grid, dim3(ROWS), 0, s, c, ldc, w.U, (long)w.ld, w.n, to_u);
}

}  // namespace skr
