/*
 * ttn_noalloc.h - allocation-free entry point of the TTN library.
 */
#ifndef TTN_NOALLOC_H
#define TTN_NOALLOC_H

#include "ttn.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of the library's static device scratch array used by ttn_qr_noalloc;
 * each GPU the library runs on holds one copy until the process ends. */
#define TTN_QR_NOALLOC_SCRATCH_BYTES ((size_t)12 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * Householder QR of ttn_debug_qr (LAPACK convention with the zero-snap of the
 * sweep's gauge shifts) on caller-owned DEVICE buffers.  The work arrays live
 * in a fixed-size device array of the library (TTN_QR_NOALLOC_SCRATCH_BYTES);
 * the call makes no device or host allocation and creates no events.
 *   rows, cols  matrix shape: 1 <= cols <= 64, rows >= cols,
 *               rows * cols < 2^31 (larger sizes are refused, TTN_E_INVALID)
 *   m           device pointer, (rows, cols) row-major complex (re, im
 *               doubles): holds M on entry and Q (rows, cols) on return
 *   r           device pointer, (cols, cols) row-major complex: receives R
 *   variant     1: one launch per column; 2: one cooperative launch with
 *               grid-wide barriers (variant 1 is taken when that grid cannot
 *               be co-resident; variant 2 cannot be captured into a graph)
 *   hip_stream  hipStream_t for the work (NULL: the null stream); the call
 *               only enqueues, results are ready when the stream is
 * The scratch is shared by every call on a GPU and keeps the last call's
 * contents; each call clears the counters it needs.  Calls that overlap on one
 * GPU (other streams, other threads) race and give wrong results.
 * Errors: TTN_E_INVALID (shape, null pointer, variant), TTN_E_DEVICE (HIP
 * error); ttn_qr_noalloc_last_error() returns the message (this thread). */
ttn_status ttn_qr_noalloc(int64_t rows, int32_t cols, void *m, void *r, int32_t variant, void *hip_stream);
const char *ttn_qr_noalloc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TTN_NOALLOC_H */
