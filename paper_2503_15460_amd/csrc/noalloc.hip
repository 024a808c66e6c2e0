// Allocation-free QR entry point: the Householder QR kernels of the sweep's
// gauge shifts on caller-owned device buffers, with their work arrays in a
// fixed-size device array of the library instead of hipMalloc'd memory.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "kernels.h"
#include "ttn.h"
#include "ttn_internal.h"
#include "ttn_noalloc.h"

namespace ttn {

// Work arrays of the many-work-group and cooperative QR kernels, carved from
// `scratch` in 256-byte aligned pieces (sizes as the sweep engine allocates).
namespace {
constexpr size_t al(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t QW_TAU = al(16 * 64), QW_SCL = al(16 * 64), QW_DIAG = al(16 * 64), QW_SNAP = al(4 * 64),
                 QW_W = al(16 * 64 * 64), QW_ROWI = al(16 * 64), QW_PART = al(8 * QRM_BLOCKS_MAX * (2 + 2 * 64)),
                 QW_S = al(16 * (size_t)QRM_BLOCKS_MAX * 64 * 63 / 2), QW_K = al(16 * 64 * 64), QW_THR = al(8 * 4),
                 QW_CNT = al(4 * 4), QW_CPART = al(8 * 2 * (size_t)QRM_BLOCKS_MAX * QRC_REC), QW_BAR = al(4 * 192);
constexpr size_t QW_TOTAL = QW_TAU + QW_SCL + QW_DIAG + QW_SNAP + QW_W + QW_ROWI + QW_PART + QW_S + QW_K + QW_THR +
                            QW_CNT + QW_CPART + QW_BAR;
static_assert(QW_TOTAL <= TTN_QR_NOALLOC_SCRATCH_BYTES, "QR work arrays exceed the static scratch");
}  // namespace

// One copy per GPU, held until the process ends.  In host code `scratch` is a
// host-side stand-in: its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[TTN_QR_NOALLOC_SCRATCH_BYTES];

__global__ void k_zero_words(unsigned *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// device address of `scratch` on the current device, looked up once per device
static unsigned char *scratch_ptr() {
    static std::mutex mu;
    static std::map<int, unsigned char *> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) throw Error(TTN_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    unsigned char *ptr = nullptr;
    e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        throw Error(TTN_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    addr[dev] = ptr;
    return ptr;
}

static void qr_noalloc(int64_t rows, int cols, double2 *m, double2 *r, int variant, hipStream_t st) {
    if (!m || !r) throw Error(TTN_E_INVALID, "null device buffer");
    if (cols < 1 || cols > 64 || rows < cols)
        throw Error(TTN_E_INVALID, "QR shape out of range: need 1 <= cols <= 64 and rows >= cols");
    if (rows * (int64_t)cols >= (int64_t(1) << 31))
        throw Error(TTN_E_INVALID, "QR matrix too large: rows * cols must stay below 2^31 elements");
    if (variant != 1 && variant != 2) throw Error(TTN_E_INVALID, "variant must be 1 or 2");
    unsigned char *base = scratch_ptr();
    QRWork q{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = base + off;
        off += bytes;
        return p;
    };
    q.tau = (double2 *)take(QW_TAU);
    q.scl = (double2 *)take(QW_SCL);
    q.diag = (double2 *)take(QW_DIAG);
    q.snapped = (int *)take(QW_SNAP);
    q.w = (double2 *)take(QW_W);
    q.rowi = (double2 *)take(QW_ROWI);
    q.part = (double *)take(QW_PART);
    q.S = (double2 *)take(QW_S);
    q.K = (double2 *)take(QW_K);
    q.thr = (double *)take(QW_THR);
    q.counter = (unsigned *)take(QW_CNT);
    q.cpart = (double *)take(QW_CPART);
    q.bar = (unsigned *)take(QW_BAR);
    q.bar_base = 0;
    // the last call's contents stay behind: the ticket counter, the barrier
    // arrival counter and its failure flag must start at zero (a fill kernel,
    // so that the call can also be captured into a graph)
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, st, q.counter, 4);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, st, q.bar, 192);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(TTN_E_DEVICE, std::string("zero fill: ") + hipGetErrorString(e));
    ProfileSuspend no_profile;  // the launch profiler would create events: not here
    try {
        if (variant == 2 && launch_qr_coop(m, rows, cols, 1, r, 0, q, st)) return;
        launch_qr_multi(m, rows, cols, 1, r, 0, q, st);
    } catch (const Error &) {
        throw;
    } catch (const std::exception &ex) {
        throw Error(TTN_E_DEVICE, ex.what());
    }
}

}  // namespace ttn

namespace {
thread_local std::string g_noalloc_err;
}

extern "C" {

ttn_status ttn_qr_noalloc(int64_t rows, int32_t cols, void *m, void *r, int32_t variant, void *hip_stream) {
    try {
        ttn::qr_noalloc(rows, cols, (double2 *)m, (double2 *)r, variant, (hipStream_t)hip_stream);
        return TTN_OK;
    } catch (const ttn::Error &e) {
        g_noalloc_err = e.what();
        return e.code;
    } catch (const std::exception &e) {
        g_noalloc_err = e.what();
        return TTN_E_INVALID;
    }
}

const char *ttn_qr_noalloc_last_error(void) { return g_noalloc_err.c_str(); }

}  // extern "C"
