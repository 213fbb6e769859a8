/*
 * gridhop_test.h - test and diagnostic switches of the grid-hopping library.
 *
 * Not needed by any caller of the hot path: every entry point of gridhop.h
 * picks its kernels and launch shapes by itself, and its results do not
 * depend on these switches beyond rounding order (the tests check that).  A
 * switch selects an alternative code path that the tests compare against the
 * default one, or forces a condition the default path only meets under
 * contention.  Nothing is read from the environment.
 *
 * State: one override per switch and per calling thread, read by the calls
 * that thread makes afterwards (at enqueue time).  Value 0 restores the
 * default.  Other threads are unaffected.
 */
#ifndef GRIDHOP_TEST_H
#define GRIDHOP_TEST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    /* gh_decision and the grid-hopping Block-OMP selections: 1 = the generic
     * one-location-per-workgroup sweep for every shape (default: the column
     * sweep wherever the slab has a power-of-two vy axis and fits LDS). */
    GH_KNOB_SWEEP_GENERIC = 1,
    /* LDS budget of a column-sweep workgroup in KiB (default 40; 8..160). */
    GH_KNOB_SWEEP_LDS_KIB = 2,
    /* Block-OMP selections after the first: 1 = maps of the residual by the
     * FFT of the residual frame (default: by linearity from the maps of the
     * frame and the fitted atoms' closed-form maps, where their tables fit). */
    GH_KNOB_BOMP_MAPS_FFT = 3,
    /* gh_refine: 1 = one workgroup per cell (default: a cluster of workgroups
     * per cell meeting at a bounded barrier in global memory). */
    GH_KNOB_REFINE_SINGLE = 4,
    /* gh_refine: frame rows per cluster workgroup, a power of two (clamped to
     * the supported splits; default: about 16 workgroups per cell). */
    GH_KNOB_REFINE_ROWS = 5,
    /* gh_refine: polls of the barrier counter before a cluster wait expires
     * (default 2^21, at least 0.2 s).  A small value makes the waits of
     * workgroups that arrive early expire, so that the NaN estimates and the
     * status count of gh_refine can be tested; every kernel still exits. */
    GH_KNOB_REFINE_SPIN_LIMIT = 6
} gh_knob;

/* Set switch `knob` for the calling thread to `value` (0: default).  Returns
 * the previous value (>= 0), or GH_EINVAL (-1) for an unknown switch or a
 * value outside the switch's range. */
int gh_test_set_knob(int32_t knob, int32_t value);

#ifdef __cplusplus
}
#endif

#endif /* GRIDHOP_TEST_H */
