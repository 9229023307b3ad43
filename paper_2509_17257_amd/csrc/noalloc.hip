// h2x_matmul_noalloc: the product of h2x_matmul with its scratch memory (x-hat,
// y-hat, the tree-ordered copy of X and the counters of the fused upward pass) in a
// file-scope device array instead of a caller workspace, for callers that cannot
// allocate device memory.  The array exists once per GPU, for the life of the
// process; its device address is looked up once per device and kept.
#include <mutex>
#include <string>

#include "device.hpp"

namespace h2x {

void set_error(const std::string &msg);

namespace {

__device__ __align__(256) char scratch[H2X_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_scratch[kMaxDevices];  // device address of `scratch` on each device, once looked up

h2x_status fail(h2x_status s, const std::string &msg) {
    set_error("h2x_matmul_noalloc: " + msg);
    return s;
}

// the current device's copy of the array (looked up on the first call on that device)
h2x_status scratch_on_current_device(char **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(H2X_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(H2X_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(H2X_EHIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch[dev] = (char *)p;
    }
    *out = g_scratch[dev];
    return H2X_OK;
}

}  // namespace
}  // namespace h2x

using namespace h2x;

extern "C" h2x_status h2x_matmul_noalloc(const h2x_mat *A, int64_t m, double alpha, const double *X, int64_t ldx,
                                         double beta, double *Y, int64_t ldy, int32_t flags, void *hip_stream) {
    if (!A || !X || !Y) return fail(H2X_EINVAL, "NULL argument");
    if (m < 1 || ldx < m || ldy < m) return fail(H2X_EINVAL, "need m >= 1, ldx >= m, ldy >= m");
    if (flags & ~H2X_TREE_ORDER) return fail(H2X_EINVAL, "unknown flags");
    if (A->dm.cplx && (m & 1))
        return fail(H2X_EINVAL, "a complex operator takes an even number of real columns");
    const int64_t n = A->dm.n;
    const char *x0 = (const char *)X, *x1 = (const char *)(X + (n - 1) * ldx + m);
    const char *y0 = (const char *)Y, *y1 = (const char *)(Y + (n - 1) * ldy + m);
    if (x0 < y1 && y0 < x1) return fail(H2X_EINVAL, "X and Y overlap");
    const size_t need = matmul_ws_bytes(A->dm, m);
    if (need > (size_t)H2X_NOALLOC_MAX_BYTES)
        return fail(H2X_ENOMEM, "the product needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                    std::to_string((size_t)H2X_NOALLOC_MAX_BYTES) +
                                    " bytes of the static array; use h2x_matmul with a workspace");
    char *ws = nullptr;
    if (h2x_status s = scratch_on_current_device(&ws)) return s;
    hipError_t e = run_matmul(A->dm, m, alpha, X, ldx, beta, Y, ldy, (flags & H2X_TREE_ORDER) != 0, ws,
                              (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(H2X_EHIP, hipGetErrorString(e));
    return H2X_OK;
}
