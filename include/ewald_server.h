/*
 * ewald_server.h -- request loop serving many independent Ewald systems on
 * one MI355X (gfx950) GPU.
 *
 * Each registered system is one plan of the evaluation in ewald.h (the
 * real-space, reciprocal-space, self and background terms of Saunders, Grant
 * & Mueller, section 3); its constant tables (k-set layout, C_k) stay
 * resident on the device between requests.  A request is one energy/force
 * evaluation of a registered system.  A native dispatcher thread owned by the
 * server takes requests in submission order and enqueues each on one of the
 * server's streams, so that small systems run beside large ones:
 *   - a system's requests start in submission order, and while one is in
 *     flight the next goes to the same stream (its plan is not re-entrant);
 *   - otherwise a small request (estimated work below that of about a
 *     5,000-ion electrolyte at the serving mix's density) goes to the express
 *     stream, stream 0, so that it never queues behind a large one, and any
 *     other request to the stream with the least outstanding estimated work
 *     among the rest (with one stream, everything goes to it);
 *   - the express stream (or the only stream) takes at most 2 launch
 *     sequences at a time and each bulk stream 1; the rest wait in the
 *     dispatcher, where a small request that arrives later still passes them;
 *   - the small requests that can start together (their workspaces fit, the
 *     express stream has a slot) go out as one batched launch sequence
 *     (ewald_energy_forces_batch: each kernel launched once over a ragged work
 *     list spanning all of them), at most 64 at a time, unless the server was
 *     made with EWALD_SERVER_FLAG_NO_BATCH;
 *   - the systems' plans run their real- and reciprocal-space chains on the
 *     request's stream (EWALD_FLAG_ONE_STREAM); requests in flight on
 *     different streams overlap instead;
 *   - with EWALD_SERVER_FLAG_EXPRESS_CUS, more than one stream and a 256-CU
 *     device, the streams are created with CU masks: the express stream runs
 *     on 16 compute units (two per XCD) and the bulk streams on the other
 *     240, so a small request never waits for the workgroups of a large one
 *     to leave a CU (throughput of large requests drops by about the share of
 *     the reserved CUs).
 * Completion is detected by polling one event per launch sequence; a request's
 * latency is measured on the server's monotonic clock from its submission to
 * the moment the dispatcher observes its completion.
 *
 * Admission by HBM footprint, per request: the server holds one device arena
 * of hbm_budget bytes; a request is started only when its per-evaluation
 * buffers (ewald_eval_workspace_bytes for its n: cell list, neighbour lists,
 * phase tables, partial sums) fit in the arena, and they return to the arena
 * when it completes.  A request that does not fit is held, not refused: it
 * starts as soon as completions free enough memory.  Later requests may start
 * before a held one while it has waited less than 20 ms; after that nothing
 * passes it.  A system whose largest request (n_max) could never fit the
 * arena is refused at registration (EWALD_ERR_ADMISSION).
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
 *   flags       0, or any of EWALD_SERVER_FLAG_EXPRESS_CUS (the express
 *               stream gets compute units of its own, see above) and
 *               EWALD_SERVER_FLAG_NO_BATCH (express requests go out one by
 *               one instead of batched).
 *   hbm_budget  bytes of the device arena for the buffers of requests in
 *               flight, allocated when the server is created; 0 means 90 % of
 *               the free device memory, at most 8 GiB. */
typedef struct {
    int32_t device;
    int32_t n_streams;
    int32_t precision;
    int32_t flags;
    uint64_t hbm_budget;
} ewald_server_params;

#define EWALD_SERVER_FLAG_EXPRESS_CUS 1
#define EWALD_SERVER_FLAG_NO_BATCH 2

/* Counters of a server (host values). */
typedef struct {
    int64_t systems;       /* registered systems                       */
    int64_t submitted;     /* requests accepted by ewald_server_submit */
    int64_t completed;     /* requests whose completion was observed   */
    int64_t in_flight;     /* enqueued on a stream, not yet completed  */
    uint64_t budget;       /* arena bytes                              */
    uint64_t used;         /* arena bytes held by requests in flight   */
    uint64_t peak_used;    /* most arena bytes held at once            */
    int64_t held;          /* requests now waiting for arena memory    */
    int64_t held_total;    /* requests that had to wait for memory     */
    int64_t masked_streams; /* bulk streams created with a CU mask     */
    int64_t batches;       /* batched launch sequences (2+ requests)  */
    int64_t batched;       /* requests those sequences carried        */
} ewald_server_stats;

/* Create a server and start its dispatcher thread.  *out is NULL on failure.
 * Errors: INVALID_ARG, DEVICE, OUT_OF_MEMORY. */
ewald_status ewald_server_create(const ewald_server_params *params, ewald_server_t *out);

/* Register a system: box side, splitting exponent, cutoffs and capacity as in
 * ewald_params (its precision, device, stream and flags fields are ignored:
 * the server's are used).  Builds the system's plan without a workspace.  On
 * success *system_id receives a non-negative id.  Errors: INVALID_ARG (bad
 * parameters), ADMISSION (a request of n_max particles could never fit the
 * arena; nothing kept), OUT_OF_MEMORY, DEVICE. */
ewald_status ewald_server_add_system(ewald_server_t server, const ewald_params *params, int32_t *system_id);

/* Wait for the system's requests, then release its plan.  Errors:
 * INVALID_ARG (unknown id). */
ewald_status ewald_server_remove_system(ewald_server_t server, int32_t system_id);

/* Submit one evaluation of a registered system; arguments as
 * ewald_energy_forces() (device pointers, n <= the system's n_max).  Returns
 * at once, also when the request has to wait for arena memory; *ticket
 * identifies the request for ewald_server_wait().  Errors (nothing
 * submitted): INVALID_ARG, CAPACITY. */
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
