// Probes (nacc_probe.h): streaming HBM read-only, write-only and copy
// kernels over 16-byte vectors, four vectors in flight per lane; the
// hardware square root and reciprocal of given inputs.
#include "common.h"
#include "nacc_probe.h"

using namespace nacc;

namespace {

constexpr int kProbeThreads = 256;
constexpr int kUnroll = 4;

__global__ void __launch_bounds__(kProbeThreads) probe_read_kernel(const uint4* __restrict__ src, int64_t n,
                                                                  uint4* __restrict__ dst) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kProbeThreads;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kProbeThreads + threadIdx.x;
    uint32_t acc = 0;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        uint4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n; i += stride) {
        const uint4 v = src[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9E3779B9u) dst[0] = make_uint4(acc, acc, acc, acc);
}

__global__ void __launch_bounds__(kProbeThreads) probe_write_kernel(uint4* __restrict__ dst, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kProbeThreads;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kProbeThreads + threadIdx.x;
    const uint4 z = make_uint4(0, 0, 0, 0);
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) dst[i + u * stride] = z;
    }
    for (; i < n; i += stride) dst[i] = z;
}

__global__ void __launch_bounds__(kProbeThreads) probe_copy_kernel(const uint4* __restrict__ src,
                                                                  uint4* __restrict__ dst, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kProbeThreads;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kProbeThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        uint4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) dst[i + u * stride] = v[u];
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

__global__ void __launch_bounds__(kProbeThreads) probe_sqrt_rcp_kernel(const float* __restrict__ x, int64_t n,
                                                                       float* __restrict__ s, float* __restrict__ r) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kProbeThreads + threadIdx.x;
    if (i < n) {
        s[i] = __builtin_amdgcn_sqrtf(x[i]);
        r[i] = __builtin_amdgcn_rcpf(x[i]);
    }
}

}  // namespace

extern "C" int nacc_probe_fast_sqrt_rcp(const float* x, int64_t n, float* sqrt_out, float* rcp_out, void* stream) {
    clear_error();
    NACC_REQUIRE(n >= 0 && n <= INT32_MAX, NACC_EINVAL, "n = %lld out of [0, 2^31 - 1]",
                 static_cast<long long>(n));
    NACC_REQUIRE(n == 0 || (x != nullptr && sqrt_out != nullptr && rcp_out != nullptr), NACC_EINVAL,
                 "x, sqrt_out and rcp_out must be non-NULL");
    if (n == 0) return NACC_OK;
    hipLaunchKernelGGL(probe_sqrt_rcp_kernel, dim3(static_cast<unsigned>((n + kProbeThreads - 1) / kProbeThreads)),
                       dim3(kProbeThreads), 0, as_stream(stream), x, n, sqrt_out, rcp_out);
    return check_launch("probe sqrt rcp");
}

extern "C" int nacc_probe_hbm(int32_t kind, const void* src, void* dst, int64_t n_bytes, int32_t blocks,
                              void* stream) {
    clear_error();
    NACC_REQUIRE(kind >= NACC_PROBE_READ && kind <= NACC_PROBE_COPY, NACC_EINVAL, "kind = %d unknown", kind);
    NACC_REQUIRE(n_bytes > 0 && n_bytes % 16 == 0, NACC_EINVAL,
                 "n_bytes = %lld must be a positive multiple of 16", static_cast<long long>(n_bytes));
    NACC_REQUIRE(blocks >= 1 && blocks <= (1 << 20), NACC_EINVAL, "blocks = %d not in [1, 2^20]", blocks);
    NACC_REQUIRE(dst != nullptr, NACC_EINVAL, "dst must be non-NULL");
    NACC_REQUIRE(kind == NACC_PROBE_WRITE || src != nullptr, NACC_EINVAL, "src must be non-NULL");
    NACC_REQUIRE(reinterpret_cast<uintptr_t>(dst) % 16 == 0 && reinterpret_cast<uintptr_t>(src) % 16 == 0,
                 NACC_EINVAL, "src and dst must be 16-byte aligned");
    if (kind == NACC_PROBE_COPY) {
        const auto a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
        const auto n = static_cast<uintptr_t>(n_bytes);
        NACC_REQUIRE(a + n <= b || b + n <= a, NACC_EINVAL, "src and dst overlap");
    }
    const int64_t n = n_bytes / 16;
    hipStream_t s = as_stream(stream);
    const dim3 grid(static_cast<unsigned>(blocks)), block(kProbeThreads);
    if (kind == NACC_PROBE_READ) {
        hipLaunchKernelGGL(probe_read_kernel, grid, block, 0, s, static_cast<const uint4*>(src), n,
                           static_cast<uint4*>(dst));
    } else if (kind == NACC_PROBE_WRITE) {
        hipLaunchKernelGGL(probe_write_kernel, grid, block, 0, s, static_cast<uint4*>(dst), n);
    } else {
        hipLaunchKernelGGL(probe_copy_kernel, grid, block, 0, s, static_cast<const uint4*>(src),
                           static_cast<uint4*>(dst), n);
    }
    return check_launch("hbm probe");
}
