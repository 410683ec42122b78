/*
 * pp_server.h -- persistent request loop for pressure solves of independent cases.
 *
 * Serves the step-11 pressure solve (Kumar & Vanka, arXiv 2104.01636,
 * Section 2.2) for many independent duct cases of uneven sizes on one GPU.  A
 * case keeps its solver handle, multigrid hierarchy and last pressure resident
 * on the device between requests: a request without a new density skips the
 * set-up, and every solve is warm-started from the case's previous pressure.
 *
 * Requests queue in arrival order.  A free slot (worker thread) takes the
 * first queued request whose case is idle and whose device footprint fits the
 * budget, evicting idle cases least-recently-used first when that makes room.
 * Slots run concurrently, each case on its own HIP stream, so requests that
 * arrive while others run are admitted as slots and memory free up and their
 * kernels overlap on the device.  Results do not depend on what else runs:
 * every reduction has a fixed order.
 *
 * Ownership: the caller keeps rho, rhs and p_out (device pointers) valid and
 * unchanged until pp_server_wait reports the request done.  The server owns the
 * cases.  All functions are thread-safe.
 */
#ifndef PP_SERVER_H
#define PP_SERVER_H

#include <stddef.h>

#include "pp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pp_server_s* pp_server;

typedef struct {
    size_t budget_bytes; /* device bytes all resident cases may hold together (> 0) */
    int slots;           /* concurrent solves, 1..64 */
} pp_server_config;

/* Device work of one case.  NULL backend = the HIP library (pp_create with a
 * stream per case, resident pressure, device-to-device copy into p_out).  A
 * host backend lets the scheduler run without a GPU.  Each function returns a
 * pp_status; footprint returns 0 for an invalid configuration. */
typedef struct {
    void* ctx;
    size_t (*footprint)(void* ctx, const pp_config* cfg);
    int (*open_case)(void* ctx, const pp_config* cfg, void** case_state);
    int (*set_density)(void* ctx, void* case_state, const double* rho);
    int (*solve)(void* ctx, void* case_state, const double* rhs, double* p_out, pp_stats* st);
    void (*close_case)(void* ctx, void* case_state);
    const char* (*error)(void* ctx, void* case_state);
} pp_backend;

typedef struct {
    int status;        /* pp_status of the request */
    pp_stats stats;
    double t_submit, t_start, t_end;  /* seconds, steady clock */
    double latency_ms; /* t_end - t_submit */
    int new_density;   /* the request carried a density (set-up ran) */
    char message[160];
} pp_request_result;

typedef struct {
    long long completed, succeeded, rejected, queued;
    int running, max_running;
    long long resident_cases;
    size_t resident_bytes, peak_resident_bytes;
    long long evictions;
    double latency_p50_ms, latency_p99_ms, latency_max_ms; /* successful requests, submit to result */
    double solves_per_s;                                   /* successes / (last result - first submit) */
} pp_server_stats;

/* Start the slots.  backend may be NULL (HIP library). */
int pp_server_create(const pp_server_config* cfg, const pp_backend* backend, pp_server* out);

/* Queue one solve of case case_id (grid and mode from cfg; the tolerance and
 * iteration cap of a case are those of its first request).  rho: the case's
 * new density, or NULL to keep the resident one (the first request of a case
 * must bring one).  rhs: right-hand side; p_out: receives the pressure (may be
 * NULL).  Returns at once with *req_id. */
int pp_server_submit(pp_server s, long long case_id, const pp_config* cfg, const double* rho, const double* rhs,
                     double* p_out, long long* req_id);

/* Wait for a request (timeout_s < 0: no limit).  Returns PP_OK when done (the
 * request's own status is in out->status), 1 on time-out. */
int pp_server_wait(pp_server s, long long req_id, double timeout_s, pp_request_result* out);

int pp_server_get_stats(pp_server s, pp_server_stats* out);

/* Drain queued and running requests, stop the slots, release every case. */
int pp_server_destroy(pp_server s);

const char* pp_server_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PP_SERVER_H */
