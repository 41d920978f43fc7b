// Internal helpers of the gfx950 library: error reporting, launch checks and
// wave64 cross-lane primitives built on DPP (data-parallel primitives).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "nacc.h"

namespace nacc {

// Records a message for nacc_last_error() and returns `status`.
int set_error(int status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// Clears the calling thread's message.
void clear_error();
// Converts a pending launch error into NACC_EHIP.
int check_launch(const char* what);
// Launch parameters picked by the caller or the autotuner (nacc_set_tuning).
const nacc_tuning& tuning();

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Per-axis scale fl32(res / (hi - lo)): the quotient in FP64, rounded once.
inline float axis_scale(int res, float lo, float hi) {
    return static_cast<float>(static_cast<double>(res) /
                              (static_cast<double>(hi) - static_cast<double>(lo)));
}

constexpr int kWave = 64;
constexpr int kWaveLog2 = 6;

// Layout of the skip buffer of nacc_grid_build_skip for grids of res^3
// cells (res % 4 == 0): the distance field (one byte per coarse cell of
// 4^3 fine cells, per grid), scratch of its build of the same size, then,
// 256-byte aligned, the halo bits: per grid one bit per cell of 2^3 fine
// cells (C order, LSB first, rounded up to whole 64-bit words), set when an
// occupied fine cell lies within kHaloReach fine cells (on every axis) of it.
constexpr int kHaloReach = 2;

__host__ __device__ inline int64_t skip_field_cells(int res) {
    const int64_t c = res / 4;
    return c * c * c;
}

__host__ __device__ inline int64_t halo_offset(int res, int n_grids) {
    return ((2 * skip_field_cells(res) * n_grids + 255) / 256) * 256;
}

// 32-bit words of one grid's halo bits.
__host__ __device__ inline int64_t halo_words(int res) {
    const int64_t h = res / 2;
    return ((h * h * h + 63) / 64) * 2;
}

}  // namespace nacc

#define NACC_REQUIRE(cond, status, ...)                    \
    do {                                                   \
        if (!(cond)) return ::nacc::set_error(status, __VA_ARGS__); \
    } while (0)

// ---------------------------------------------------------------------------
// Device side.  Every helper below must be called with all 64 lanes active
// (wave-uniform control flow): DPP reads the registers of neighbouring lanes.
// ---------------------------------------------------------------------------
namespace nacc {
namespace dev {

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) {
    return __builtin_amdgcn_ballot_w64(p);
}

// Orders one wave's LDS writes before its later reads of other lanes' slots
// (and those reads before the slots are written again): a wave-scope fence
// pair around a wave barrier.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Logical index of workgroup b of a grid of n.  The hardware hands
// workgroups to the 8 XCDs in turn (b mod 8), each XCD with its own L2;
// renumbered here so that every XCD takes runs of G consecutive logical
// workgroups (runs interleaved over the XCDs every 8 G workgroups), data
// shared by neighbouring workgroups (cache lines at the ends of their
// ranges) is fetched by one L2 instead of two, while uneven costs along the
// index still spread over all XCDs.  A bijection of [0, n): the tail past
// the last whole period keeps its index.
template <int G>
__device__ __forceinline__ int64_t xcd_grouped(int64_t b, int64_t n) {
    constexpr int64_t kXcds = 8, kPeriod = kXcds * G;
    if (b >= (n / kPeriod) * kPeriod) return b;
    const int64_t base = (b / kPeriod) * kPeriod, i = b - base;
    return base + (i % kXcds) * G + i / kXcds;
}

// Number of set bits of `mask` below the calling lane.
__device__ __forceinline__ int bits_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

template <typename T>
__device__ __forceinline__ T uniform(T v);

template <>
__device__ __forceinline__ int uniform<int>(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <>
__device__ __forceinline__ float uniform<float>(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

__device__ __forceinline__ float read_lane(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

__device__ __forceinline__ double read_lane(double v, int lane) {
    uint64_t b = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffu), lane);
    uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ __forceinline__ int read_lane(int v, int lane) {
    return __builtin_amdgcn_readlane(v, lane);
}

// DPP move with 0 written into lanes whose source is out of range or masked.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, false));
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp(double v) {
    uint64_t b = __builtin_bit_cast(uint64_t, v);
    int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffu), CTRL, ROW_MASK, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint32_t>(lo));
}

// DPP controls (GFX9 encoding).
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowShl1 = 0x101, kRowShl2 = 0x102, kRowShl4 = 0x104, kRowShl8 = 0x108;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143, kWaveShr1 = 0x138, kWaveShl1 = 0x130;

// Inclusive prefix sum across the 64 lanes: Hillis-Steele within each row of
// 16 lanes, then the row totals are carried by two row broadcasts.  The
// association order is fixed, so results are deterministic.
template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T x) {
    x = x + dpp<kRowShr1>(x);
    x = x + dpp<kRowShr2>(x);
    x = x + dpp<kRowShr4>(x);
    x = x + dpp<kRowShr8>(x);
    x = x + dpp<kRowBcast15, 0xa>(x);
    x = x + dpp<kRowBcast31, 0xc>(x);
    return x;
}

// The value of the lane below (0 in lane 0).
template <typename T>
__device__ __forceinline__ T shift_up_one(T x) {
    return dpp<kWaveShr1>(x);
}

// The value of the lane above (0 in lane 63).
template <typename T>
__device__ __forceinline__ T shift_down_one(T x) {
    return dpp<kWaveShl1>(x);
}

// Inclusive suffix sum across the 64 lanes (lane i gets the sum over lanes
// i..63): Hillis-Steele within each row of 16 lanes towards lower lanes,
// then each row adds the totals of the rows above it.  Fixed association.
template <typename T>
__device__ __forceinline__ T wave_inclusive_suffix(T x) {
    x = x + dpp<kRowShl1>(x);
    x = x + dpp<kRowShl2>(x);
    x = x + dpp<kRowShl4>(x);
    x = x + dpp<kRowShl8>(x);
    const T r1 = read_lane(x, 16), r2 = read_lane(x, 32), r3 = read_lane(x, 48);
    const T above2 = r3;
    const T above1 = r2 + r3;
    const T above0 = r1 + above1;
    const int row = lane_id() >> 4;
    const T add = row == 0 ? above0 : (row == 1 ? above1 : (row == 2 ? above2 : T(0)));
    return x + add;
}

// Sum over the 64 lanes, returned in every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
    return read_lane(wave_inclusive_sum(x), 63);
}

}  // namespace dev
}  // namespace nacc
