/*
 * mpsim_static.h -- allocation-free entry point of the block-MPS library
 * (the conventions of mpsim.h apply).
 */
#ifndef MPSIM_STATIC_H
#define MPSIM_STATIC_H

#include "mpsim.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of the static device buffer behind mps_measure_static: one copy per
 * GPU the library runs on, held until the process ends. */
#define MPS_MEASURE_STATIC_BYTES (64L << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * measurement of mps_measure (the transfer-matrix sweep of <Z_tot> and
 * <Z_tot^2>, eqs. "Z_tot" and "z2_tot") over an MPS the caller holds in
 * device memory, with its environments in a static device buffer of
 * MPS_MEASURE_STATIC_BYTES instead of buffers the library allocates. It
 * calls no allocation routine, copies nothing between host and device and
 * does not synchronise.
 *
 *   nsites     number of sites N >= 1
 *   bonds      host array of N + 1 bond dimensions, bonds[0] = bonds[N] = 1
 *   dims       host array of N local dimensions, each 2, 4, 8 or 16 (2^w
 *              fused qubits, the first qubit the most significant bit)
 *   sites      host array of N device pointers; site p is the row-major
 *              (bonds[p] dims[p]) x bonds[p+1] matrix of interleaved
 *              complex128 values, in any gauge (the sweep does not use the
 *              canonical form); read only
 *   hip_stream the hipStream_t the work is enqueued on (NULL: null stream)
 *   out_dev    device pointer to 3 doubles, written on the stream:
 *              <psi|psi>, <Z_tot>/n and <Z_tot^2>/n^2 (the last two divided
 *              by <psi|psi>), n = sum of w over the sites
 *
 * The buffer holds 2 x 3 b_max^2 complex environments, 3 max_p(b_p d_p
 * b_p+1) complex products and the z sums (each region 256-byte aligned);
 * an MPS whose sweep needs more returns MPS_E_UNSUPPORTED (about chi <= 256
 * at d = 16). MPS_E_INVAL for bad arguments, MPS_E_DEVICE for a HIP error;
 * messages through mps_last_error(NULL). Every call on a GPU uses that
 * GPU's one buffer, which keeps the last call's contents (each call writes
 * every region it reads before reading it): calls that overlap in time on
 * one GPU (unordered streams, several threads) race. */
mps_status mps_measure_static(int32_t nsites, const int32_t* bonds, const int32_t* dims,
                              const void* const* sites, void* hip_stream, double* out_dev);

#ifdef __cplusplus
}
#endif
#endif /* MPSIM_STATIC_H */
