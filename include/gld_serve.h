/*
 * gld_serve.h -- C ABI of libgld's continuous-batching server: GLD trajectory
 * requests (a system of gld.h, an initial state and a number of steps) that
 * arrive over time are admitted into one batch (include/gld_batch.h) as a
 * system slot and a workspace piece of their footprint free up, first come
 * first served; every admitted request keeps its state on the device and all
 * of them advance together, chunk by chunk, until each has run its steps.
 * A request's result does not depend on the others it shared the GPU with:
 * each system of a batch computes in an order fixed by itself.
 */
#ifndef GLD_SERVE_H
#define GLD_SERVE_H

#include "gld_batch.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gld_server gld_server;

typedef struct {
    int64_t id;
    int64_t n;            /* particles                                            */
    int32_t m_max;
    int32_t status;       /* GLD_OK, or the latched device error of the system    */
    int64_t steps;
    size_t footprint;     /* device bytes the request took in the batch           */
    double arrival_s;     /* seconds from gld_server_run's start                  */
    double admitted_s;    /* when it was placed in the batch (-1: not yet)        */
    double done_s;        /* when its last step completed (-1: not yet)           */
} gld_request_info;

/* A server over a batch of at most max_systems systems in the caller's
 * workspace and stream; requests advance chunk_steps steps per batch launch
 * (fewer when one finishes earlier).  schedule may be NULL (the batch's
 * default lane thresholds). */
gld_status gld_server_create(int32_t precision, int32_t max_systems, void *d_workspace, size_t workspace_bytes,
                             void *hip_stream, int32_t chunk_steps, const gld_batch_schedule *schedule,
                             gld_server **out);

/* Queue a request arriving arrival_s seconds after gld_server_run starts.
 * Its one-off host construction (noise filters, noise interval) runs here;
 * *footprint receives its device bytes.  Inputs are copied. */
gld_status gld_server_submit(gld_server *sv, const gld_params *params, const double *r0, const double *v0,
                             int64_t steps, double arrival_s, int64_t *id, size_t *footprint);

/* Serve every queued request: admit on arrival as room frees up, step all
 * admitted requests together, retire each after its steps (its final state
 * copied to the host).  Returns when all are done; waits (sleeps) for
 * arrivals while nothing is admitted. */
gld_status gld_server_run(gld_server *sv);

/* Timings of a request and (out may be NULL) its final state: r, v, f_c,
 * f_d, f_r as gld_read_state gives them (the history is not kept). */
gld_status gld_server_request(const gld_server *sv, int64_t id, gld_request_info *info, gld_state *out);

/* Wall time of the last gld_server_run and the batch steps it launched. */
gld_status gld_server_stats(const gld_server *sv, double *makespan_s, int64_t *batch_steps);

gld_status gld_server_destroy(gld_server *sv);

#ifdef __cplusplus
}
#endif

#endif /* GLD_SERVE_H */
