// Pinned host staging for the library's host-to-device list uploads (box lists,
// tile lists, norm and restriction lists, slot tables).
//
// A copy from pageable host memory makes the host wait until the device has
// executed everything queued before it; each such wait leaves the GPU idle for a
// host round trip.  Lists are therefore written into pinned buffers, uploaded
// with hipMemcpyAsync and an event recorded behind the copy; a buffer is handed
// out again only once its event has completed, so calls return without waiting
// for the device.  The pool grows to the number of uploads in flight at once
// (64 KiB and up per buffer) and keeps its buffers until the process ends.
#include <mutex>
#include <vector>

#include "sgw_api_internal.h"

namespace {

struct Buf {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr; // recorded behind the last copy that read the buffer
    int device = -1;
    bool reserved = false;     // handed out, copy not yet enqueued
    bool pending = false;      // a copy that reads it may still run
};

std::mutex g_mu;
std::vector<Buf> g_bufs;

} // namespace

hipError_t staging_acquire(size_t bytes, int* handle, void** host)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_mu);
    int best = -1;
    for (int i = 0; i < (int)g_bufs.size(); i++) {
        Buf& b = g_bufs[i];
        if (b.reserved || b.device != dev || b.bytes < bytes) continue;
        if (b.pending) {
            const hipError_t q = hipEventQuery(b.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return q;
            b.pending = false;
        }
        if (best < 0 || b.bytes < g_bufs[best].bytes) best = i;
    }
    if (best < 0) {
        Buf b;
        size_t sz = 64 * 1024;
        while (sz < bytes) sz *= 2;
        e = hipHostMalloc(&b.host, sz, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipHostFree(b.host);
            return e;
        }
        b.bytes = sz;
        b.device = dev;
        g_bufs.push_back(b);
        best = (int)g_bufs.size() - 1;
    }
    g_bufs[best].reserved = true;
    *handle = best;
    *host = g_bufs[best].host;
    return hipSuccess;
}

hipError_t staging_upload(int handle, size_t offset, void* dst_dev, size_t bytes, hipStream_t s)
{
    void* src = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        src = (unsigned char*)g_bufs[handle].host + offset;
    }
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst_dev, src, bytes, hipMemcpyHostToDevice, s);
}

hipError_t staging_release(int handle, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Buf& b = g_bufs[handle];
    b.reserved = false;
    const hipError_t e = hipEventRecord(b.done, s);
    if (e != hipSuccess) {
        // the copies may still read the buffer: wait for them before it is reused
        (void)hipStreamSynchronize(s);
        b.pending = false;
        return e;
    }
    b.pending = true;
    return hipSuccess;
}

void staging_cancel(int handle)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_bufs[handle].reserved = false;
}
