// The error norms of many solves without any allocation (sgw_norms_many_static).
//
// sgw_norms_many takes its pair list and partial sums in a caller-passed scratch
// buffer and uploads the list through pinned staging.  Callers that cannot
// allocate (graph capture, tight serving loops) get the same kernels over a
// file-scope device array instead: the pair list travels to the device as the
// argument of one small kernel, which writes it into the array, and the partial
// sums follow it there.  Each device holds its own copy of the array; host code
// reaches it only through the address hipGetSymbolAddress returns for that
// device, taken once per device while it is current.
#include <mutex>

#include "sgw_api_internal.h"

#define SGW_STATIC_MAX_PAIRS 32
#define SGW_STATIC_ITEMS_BYTES 2048  // >= SGW_STATIC_MAX_PAIRS * sizeof(NormItem), 256-byte multiple
#define SGW_STATIC_PARTIALS_BYTES ((size_t)SGW_STATIC_MAX_PAIRS * 2 * SGW_NPART * sizeof(double))
#define SGW_STATIC_SCRATCH_BYTES (SGW_STATIC_ITEMS_BYTES + SGW_STATIC_PARTIALS_BYTES)
#define SGW_STATIC_MAX_DEVICES 64

static_assert(SGW_STATIC_MAX_PAIRS * sizeof(NormItem) <= SGW_STATIC_ITEMS_BYTES, "pair list does not fit");

namespace {

static __device__ __align__(256) unsigned char scratch[SGW_STATIC_SCRATCH_BYTES];

struct NormPack {
    NormItem item[SGW_STATIC_MAX_PAIRS];
    int32_t n;
};

// one thread per pair: the list from the kernel argument into device memory
__global__ void put_norm_items_kernel(NormPack pack, NormItem* dst)
{
    const int i = threadIdx.x;
    if (i < pack.n) dst[i] = pack.item[i];
}

std::mutex g_mu;
void* g_ptr[SGW_STATIC_MAX_DEVICES] = {};

// The device address of `scratch` on the current device, looked up the first time.
hipError_t scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SGW_STATIC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

} // namespace

extern "C" uint64_t sgw_norms_many_static_max_bytes(void) { return SGW_STATIC_SCRATCH_BYTES; }

extern "C" sgw_status sgw_norms_many_static(sgw_solver_t* const* solvers, const double* const* a,
                                            const double* const* b, int32_t n, double* result_dev,
                                            void* hip_stream)
{
    if (!solvers || !a || !b || n <= 0 || !result_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    if (n > SGW_STATIC_MAX_PAIRS)
        return sgw_fail(SGW_ERR_INVALID_ARG, "at most %d pairs per call without allocation, %d given",
                        SGW_STATIC_MAX_PAIRS, n);
    NormPack pack;
    pack.n = n;
    int mp = 1;
    for (int i = 0; i < n; i++) {
        if (!solvers[i] || !a[i] || !b[i]) return sgw_fail(SGW_ERR_INVALID_ARG, "null solver or array %d", i);
        const int64_t cnt = solvers[i]->plan->fine_nodes;
        const int parts = norms_parts(cnt);
        pack.item[i] = NormItem{a[i], b[i], cnt, result_dev + 2 * (size_t)i, parts, 0};
        mp = parts > mp ? parts : mp;
    }
    for (int i = n; i < SGW_STATIC_MAX_PAIRS; i++) pack.item[i] = NormItem{};
    // the partial sums of pair i start at 2 mp i doubles: within the array for n <= the maximum
    if ((size_t)n * 2 * mp * sizeof(double) > SGW_STATIC_PARTIALS_BYTES)
        return sgw_fail(SGW_ERR_UNSUPPORTED, "partial sums exceed the static scratch");
    void* base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return sgw_hip_fail(e, "static scratch address");
    NormItem* items = (NormItem*)base;
    double* partials = (double*)((unsigned char*)base + SGW_STATIC_ITEMS_BYTES);
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(put_norm_items_kernel, dim3(1), dim3(SGW_STATIC_MAX_PAIRS), 0, st, pack, items);
    e = hipGetLastError();
    if (e != hipSuccess) return sgw_hip_fail(e, "pair list");
    e = launch_norms_many(items, n, mp, partials, st);
    if (e != hipSuccess) return sgw_hip_fail(e, "norms many (static scratch)");
    return SGW_OK;
}
