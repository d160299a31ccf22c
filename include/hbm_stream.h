/*
 * hbm_stream.h - plain HBM streaming kernels (libhbmstream.so), a
 * measurement aid beside the solver: the bandwidth a kernel that only
 * streams reaches on this device, the measured ceiling against which the
 * solver kernels' rates are read (the published peak being 8 TB/s).
 */
#ifndef HBM_STREAM_H
#define HBM_STREAM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { HBM_STREAM_READ = 0, HBM_STREAM_WRITE = 1, HBM_STREAM_COPY = 2 };

/* Runs one untimed and then `reps` timed launches of the streaming kernel
 * `kind` over `bytes` bytes (a multiple of 16, > 0) on `stream` (hipStream_t
 * or NULL) and writes the mean milliseconds per launch (HIP events on that
 * stream) to *ms.  Every lane moves 16 bytes per access; nt = 1 adds the
 * non-temporal hint.  blocks: workgroups of 256 lanes (grid-stride loop).
 *   READ:  src device [bytes] is read; dst (device, >= 16 bytes, 16-byte
 *          aligned) is a sink that is practically never written.
 *   WRITE: dst device [bytes] is written (src unused).
 *   COPY:  src device [bytes] is copied to dst device [bytes].
 * Both pointers 16-byte aligned.  Returns 0, 1 for a bad argument (checked
 * before any device call), 2 for a HIP error. */
int hbm_stream_run(int kind, int nt, void *dst, const void *src, size_t bytes, int blocks, int reps, void *stream,
                   float *ms);

#ifdef __cplusplus
}
#endif

#endif /* HBM_STREAM_H */
