/*
 * nacc_probe.h -- probes for measurement: HBM bandwidth, and the hardware
 * square root and reciprocal.
 *
 * NOT part of the method.  The rendering and marching kernels are bound by
 * HBM bandwidth or by vector ALU issue; to state how far each sits from the
 * bandwidth the hardware actually delivers (not only from the 8 TB/s data
 * sheet figure), these three streaming kernels measure the achievable
 * read-only, write-only and copy rates on the same device, in the manner of
 * McCalpin's STREAM benchmark.  Each moves whole 16-byte vectors with a
 * grid-stride loop, four vectors in flight per lane.
 *
 * Conventions as in nacc.h: device pointers, caller-owned memory, stream as
 * void*, status codes, nacc_last_error() for messages.
 */
#ifndef NACC_PROBE_H
#define NACC_PROBE_H

#include <stddef.h>
#include <stdint.h>

#include "nacc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Probe kinds. */
enum {
    NACC_PROBE_READ = 0,  /* read n_bytes of src; dst receives nothing unless
                             the (practically impossible) folded value of all
                             words equals a fixed constant, so the reads
                             cannot be optimised away */
    NACC_PROBE_WRITE = 1, /* write n_bytes of zeros to dst */
    NACC_PROBE_COPY = 2   /* copy n_bytes from src to dst */
};

/*
 * One streaming pass of `kind` over n_bytes (a positive multiple of 16;
 * src and dst 16-byte aligned and not overlapping) with `blocks`
 * workgroups of 256 threads (1 .. 2^20).  src may be NULL for
 * NACC_PROBE_WRITE; dst must hold n_bytes for NACC_PROBE_WRITE and
 * NACC_PROBE_COPY and at least 16 bytes for NACC_PROBE_READ.
 * Errors: NACC_EINVAL for bad arguments, NACC_EHIP if the launch fails.
 */
int nacc_probe_hbm(int32_t kind, const void* src, void* dst, int64_t n_bytes,
                   int32_t blocks, void* stream);

/*
 * The hardware square root and reciprocal (v_sqrt_f32, v_rcp_f32) of n
 * floats: sqrt_out[i] and rcp_out[i] for x[i] (device arrays of n floats;
 * n >= 0).  The contraction lookup decides most cells on these instructions
 * and relies on their results lying within 2 ulps of the correctly rounded
 * ones (the error bound behind its fall-back margin); this call lets that
 * be measured on the device at hand.
 * Errors: NACC_EINVAL for bad arguments, NACC_EHIP if the launch fails.
 */
int nacc_probe_fast_sqrt_rcp(const float* x, int64_t n, float* sqrt_out,
                             float* rcp_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NACC_PROBE_H */
