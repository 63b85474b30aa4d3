/*
 * ewald_server.h -- request loop serving many independent Ewald systems on
 * one MI355X (gfx950) GPU.
 *
 * Each registered system is one plan of the evaluation in ewald.h (the
 * real-space, reciprocal-space, self and background terms of Saunders, Grant
 * & Mueller, section 3); its workspace (cell lists, phase tables, structure
 * factor) stays resident on the device between requests.  A request is one
 * energy/force evaluation of a registered system.  A native dispatcher thread
 * owned by the server takes requests in submission order and enqueues each on
 * one of the server's streams, so that small systems run beside large ones:
 *   - a system's requests are serialised (they share its workspace): while one
 *     is in flight, the next goes to the same stream;
 *   - otherwise the stream with the least outstanding work (estimated from N
 *     and the k-set size) is taken.
 * Completion is detected by polling one event per request; the request's
 * latency is measured on the server's monotonic clock from its submission to
 * the moment the dispatcher observes its completion.
 *
 * Admission: a system is admitted only if its plan workspace
 * (ewald_plan_workspace_bytes) fits the budget still free; nothing is
 * allocated otherwise (EWALD_ERR_ADMISSION).
 *
 * Thread safety: every entry point may be called from any host thread.  The
 * caller guarantees that a request's inputs are complete on the device when
 * it is submitted (e.g. its producing stream was synchronised) and reads its
 * outputs only after ewald_server_wait() returned for it.  Results of a
 * request are identical, bit for bit, to those of ewald_energy_forces() on a
 * plan with the same parameters, alone or in any mix.
 */
#ifndef EWALD_MI355X_SERVER_H
#define EWALD_MI355X_SERVER_H

#include <stddef.h>
#include <stdint.h>

#include "ewald.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ewald_server_s *ewald_server_t;

/* Server parameters.
 *   device      HIP device ordinal.
 *   n_streams   streams requests are spread over, 1 <= n_streams <= 16.
 *   precision   EWALD_PRECISION_FP64 or EWALD_PRECISION_MIXED, for every system.
 *   flags       reserved, must be 0.
 *   hbm_budget  bytes of plan workspace the server may hold; 0 means 90 % of
 *               the device memory free when the server is created. */
typedef struct {
    int32_t device;
    int32_t n_streams;
    int32_t precision;
    int32_t flags;
    uint64_t hbm_budget;
} ewald_server_params;

/* Counters of a server (host values). */
typedef struct {
    int64_t systems;       /* registered systems                       */
    int64_t submitted;     /* requests accepted by ewald_server_submit */
    int64_t completed;     /* requests whose completion was observed   */
    int64_t in_flight;     /* enqueued on a stream, not yet completed  */
    uint64_t budget;       /* admission budget, bytes                  */
    uint64_t used;         /* workspace of the registered systems      */
} ewald_server_stats;

/* Create a server and start its dispatcher thread.  *out is NULL on failure.
 * Errors: INVALID_ARG, DEVICE, OUT_OF_MEMORY. */
ewald_status ewald_server_create(const ewald_server_params *params, ewald_server_t *out);

/* Register a system: box side, splitting exponent, cutoffs and capacity as in
 * ewald_params (its precision, device and stream fields are ignored: the
 * server's are used).  On success *system_id receives a non-negative id.
 * Errors: INVALID_ARG (bad parameters), ADMISSION (workspace above the free
 * budget; nothing allocated), OUT_OF_MEMORY, DEVICE. */
ewald_status ewald_server_add_system(ewald_server_t server, const ewald_params *params, int32_t *system_id);

/* Wait for the system's requests, release its plan and return its workspace
 * to the budget.  Errors: INVALID_ARG (unknown id). */
ewald_status ewald_server_remove_system(ewald_server_t server, int32_t system_id);

/* Submit one evaluation of a registered system; arguments as
 * ewald_energy_forces() (device pointers, n <= the system's n_max).  Returns
 * at once; *ticket identifies the request for ewald_server_wait().
 * Errors (nothing submitted): INVALID_ARG, CAPACITY. */
ewald_status ewald_server_submit(ewald_server_t server, int32_t system_id, int64_t n, const double *pos,
                                 const double *q, double *energy, double *forces, double *dEdq, int64_t *ticket);

/* Block until the request has completed, then forget the ticket (each ticket
 * is waited for exactly once).  t_submit and t_done (either may be NULL)
 * receive the submission and completion times in seconds on the server
 * clock (ewald_server_clock()).  Returns the request's status: EWALD_OK, or
 * DEVICE if its launch failed; non-finite inputs give a NaN energy and latch
 * EWALD_ERR_NONFINITE for ewald_server_system_status().  INVALID_ARG for an
 * unknown ticket. */
ewald_status ewald_server_wait(ewald_server_t server, int64_t ticket, double *t_submit, double *t_done);

/* *done = 1 if the request has completed (the ticket stays valid). */
ewald_status ewald_server_poll(ewald_server_t server, int64_t ticket, int32_t *done);

/* Block until every submitted request has completed. */
ewald_status ewald_server_drain(ewald_server_t server);

/* Wait for the system's requests, then return and clear its latched device
 * status (as ewald_plan_status()). */
ewald_status ewald_server_system_status(ewald_server_t server, int32_t system_id);

ewald_status ewald_server_get_stats(ewald_server_t server, ewald_server_stats *out);

/* The server clock: seconds of CLOCK_MONOTONIC (the clock of Python's
 * time.perf_counter() and time.monotonic() on Linux). */
double ewald_server_clock(void);

/* Drain, stop the dispatcher, release every plan and stream.  NULL is a no-op. */
void ewald_server_destroy(ewald_server_t server);

#ifdef __cplusplus
}
#endif

#endif /* EWALD_MI355X_SERVER_H */
