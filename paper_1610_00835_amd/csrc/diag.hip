// Read-rate diagnostic: the rate at which this device streams a buffer in the
// access pattern of the cached-pair products (one workgroup per contiguous
// piece, 16-byte loads, several in flight per lane).  It states the attainable
// HBM read rate beside the published peak, against which the HBM-bound
// products are judged.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"

namespace ertvie {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kUnroll = 8;

// Workgroup b reads the 16-byte words [b n16, (b + 1) n16); the sum is kept live
// and stored only when it equals a value the zero-filled buffers never produce.
__global__ __launch_bounds__(256) void k_read_pieces(const v4f* p, long n16, float never, float* sink)
{
    const v4f* q = p + (long)blockIdx.x * n16;
    float acc = 0.f;
    for (long i = threadIdx.x; i < n16; i += 256 * kUnroll) {
        v4f v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = i + 256 * u < n16 ? q[i + 256 * u] : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc += (v[u][0] + v[u][1]) + (v[u][2] + v[u][3]);
    }
    if (acc == never) sink[0] = acc;
}

}  // namespace

}  // namespace ertvie

extern "C" ert_status ert_vie_read_rate(const void* buf, size_t bytes, size_t piece, int reps, void* hip_stream,
                                        double* ms_out)
{
    using namespace ertvie;
    if (!buf || !ms_out || piece < 16 || piece % 16 != 0 || bytes < piece || reps < 1 ||
        ((uintptr_t)buf % 16) != 0) {
        record_error("ert_vie_read_rate: need a 16-byte aligned buffer, 16 <= piece <= bytes, piece a "
                     "multiple of 16, reps >= 1 and an output pointer");
        return ERT_EINVAL;
    }
    const size_t npieces = bytes / piece;
    if (npieces > 0x7fffffffu) {
        record_error("ert_vie_read_rate: too many pieces for one launch");
        return ERT_EINVAL;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    float* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ert_status st = ERT_HIPST(hipMallocAsync((void**)&sink, sizeof(float), s));
    if (st == ERT_OK) st = ERT_HIPST(hipEventCreate(&e0));
    if (st == ERT_OK) st = ERT_HIPST(hipEventCreate(&e1));
    double best = -1.0;
    for (int r = 0; st == ERT_OK && r <= reps; ++r) {   // the first pass is a warm-up
        st = ERT_HIPST(hipEventRecord(e0, s));
        if (st != ERT_OK) break;
        hipLaunchKernelGGL(k_read_pieces, dim3((unsigned)npieces), dim3(256), 0, s, (const v4f*)buf,
                           (long)(piece / 16), 12345.678f, sink);
        st = ERT_HIPST(hipGetLastError());
        if (st != ERT_OK) break;
        st = ERT_HIPST(hipEventRecord(e1, s));
        if (st == ERT_OK) st = ERT_HIPST(hipEventSynchronize(e1));
        float ms = 0.f;
        if (st == ERT_OK) st = ERT_HIPST(hipEventElapsedTime(&ms, e0, e1));
        if (st == ERT_OK && r > 0) best = best < 0 ? ms : std::min(best, (double)ms);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sink) (void)hipFreeAsync(sink, s);
    if (st == ERT_OK) *ms_out = best;
    return st;
}
