// cg_solve_async_noalloc: the stream-ordered solve without any device
// allocation.  Its workspace (the Krylov vectors, the block partials and
// the device result record) lives in one file-scope device array, sized for
// systems of up to kNoAllocMaxRows rows; the array is part of the library's
// code object, so every GPU the library runs on holds its own copy from
// module load until the process ends.
//
// Host code never uses the array's name as an address (on the host it is a
// stand-in, not a device pointer): its device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and that
// address is what the kernels receive.
#include <cstring>
#include <mutex>

#include "host.h"

namespace fs {
namespace {

constexpr int64_t kNoAllocMaxRows = int64_t(1) << 18;   // 262,144 rows
// doubles: 7 vectors of the largest system, the block partials and the
// barrier counter, and the result record rounded up to whole doubles
constexpr int64_t kInfoDoubles =
    (int64_t(sizeof(fs_cg_info)) + int64_t(sizeof(double)) - 1) /
    int64_t(sizeof(double));
constexpr int64_t kScratchDoubles =
    7 * kNoAllocMaxRows + kPersistPartials + kInfoDoubles;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the device must be
// current); looked up on the first call on each device.
fs_status scratch_address(int device, double **out)
{
    if (device < 0 || device >= kMaxDevices)
        return set_error(FS_E_ARG, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(FS_E_HIP, "hipGetSymbolAddress(scratch): %s",
                             hipGetErrorString(e));
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[device];
    return FS_OK;
}

}  // namespace
}  // namespace fs

using namespace fs;

extern "C" fs_status cg_solve_async_noalloc(fs_csr_t A, const double *b,
                                            double *x, const fs_cg_opts *opts,
                                            fs_cg_info *info, hipStream_t s)
{
    fs_cg_opts o;
    FS_TRY(async_check(A, b, x, opts, info, o));
    if (A->n_rows > kNoAllocMaxRows)
        return set_error(FS_E_ARG,
                         "%d rows: the allocation-free solve holds systems of "
                         "up to %lld rows", A->n_rows,
                         static_cast<long long>(kNoAllocMaxRows));
    if (A->n_rows == 0) {
        std::memset(info, 0, sizeof(fs_cg_info));
        return FS_OK;
    }
    DeviceGuard g(A->device);
    double *base = nullptr;
    FS_TRY(scratch_address(A->device, &base));
    double *ws = base;                         // 7 n doubles
    double *part = base + 7 * kNoAllocMaxRows; // kPersistPartials doubles
    fs_cg_info *dinfo =
        reinterpret_cast<fs_cg_info *>(part + kPersistPartials);
    return async_enqueue(A, b, x, o, ws, part, dinfo, info, s);
}
