/*
 * npm_serve.h -- serving form of libnpm: many guiding sessions resident on one
 * MI355X, their requests batched continuously into persistent kernels.
 *
 * Each session is an independent guiding network (its own grid, MLP and Adam
 * state; a context of npm.h).  A path tracer renders many images at once,
 * each online-training its own network (Sec. 5.2: one optimisation step per
 * sample per pixel, queries at every bounce); the server takes their query
 * and training batches as they arrive and runs them as rounds.  A round is
 * formed while the previous one is still on the GPU, so the device stays
 * busy; every request admitted to a round shares the round's persistent
 * kernels with the other sessions' requests (tiles of 32 vertices, any
 * session, in one launch), followed by the Adam step of every session that
 * trained in the round.
 *
 * Ordering: requests of one session take effect in submission order -- a
 * query submitted after a training batch sees the updated weights; a round
 * holds at most one training batch per session, after that session's
 * earlier queries.  Different sessions are independent.
 *
 * Admission: a session is created only if its persistent device memory fits
 * the server's HBM budget (NPM_ERR_BUDGET otherwise); a round takes requests
 * in arrival order up to the round's vertex capacity (a request larger than
 * the capacity runs in a round of its own); the rest wait for a later round.
 *
 * All request buffers are caller-owned DEVICE pointers in the layouts of
 * npm_query / npm_backward, and must stay valid until npm_wait returns for
 * the request.  Every call returns an npm_status and sets npm_last_error().
 */
#ifndef NPM_SERVE_H
#define NPM_SERVE_H

#include "npm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct npm_server npm_server;

typedef struct {
    int64_t budget_bytes;    /* HBM budget for resident sessions (> 0)           */
    int32_t max_sessions;    /* session slots, 1..256                            */
    int32_t round_vertices;  /* vertex capacity of one round (>= 1024)           */
    int32_t plain_path;      /* 1: run every request through its session's own
                                npm_query / npm_train_step calls instead of the
                                shared persistent kernels (the per-session path) */
    int32_t reserved;
} npm_server_config;

typedef struct {
    double submit_us;        /* host clock (microseconds) at submission           */
    double launch_us;        /* host clock when its round was launched            */
    double done_us;          /* host clock when its round was seen complete       */
    int64_t round;           /* round number                                      */
    int64_t n;               /* vertices                                          */
    int32_t kind;            /* 0 query, 1 train                                  */
    int32_t session;
} npm_request_info;

typedef struct {
    int64_t rounds;
    int64_t requests_done;
    int64_t vertices_done;
    int64_t sessions;
    int64_t bytes_in_use;    /* persistent device memory of resident sessions   */
    double busy_us;          /* sum over rounds of launch-to-completion time      */
} npm_server_stats;

/* Creates a server on the current device with its own HIP stream and
 * scheduler thread.                                                        */
npm_status npm_server_create(const npm_server_config *cfg, npm_server **out);
/* Finishes every submitted request, then frees all sessions.  NULL is a no-op. */
npm_status npm_server_destroy(npm_server *srv);

/* Creates a session from *cfg (the shared persistent kernels take the
 * precision form, NPM_PREC_BF16; other configurations are served through
 * the per-session path).  NPM_ERR_BUDGET if it does not fit.              */
npm_status npm_session_create(npm_server *srv, const npm_config *cfg, int32_t *sid);
/* Waits for the session's requests, then frees it.                        */
npm_status npm_session_destroy(npm_server *srv, int32_t sid);
/* The session's context, e.g. for npm_get_state; not to be used for hot-path
 * calls while the server runs.                                             */
npm_status npm_session_ctx(npm_server *srv, int32_t sid, npm_ctx **ctx);

/* Enqueues a query (as npm_query) or a training batch (as npm_train_step;
 * stats_out: device pointer to two doubles, loss and squared gradient norm,
 * or NULL).  *req receives the request id.                                 */
npm_status npm_submit_query(npm_server *srv, int32_t sid, int64_t n, const float *pos,
                            const float *dir, uint64_t rng_seed, uint32_t rng_stream,
                            float *lobes, float *pdf, float *sample_dir, float *sample_pdf,
                            uint64_t *req);
npm_status npm_submit_train(npm_server *srv, int32_t sid, int64_t n, const float *pos,
                            const float *dir, const float *radiance, const float *sampling_pdf,
                            double *stats_out, uint64_t *req);

/* hold != 0: the server forms no new round (rounds already launched
 * finish); requests submitted meanwhile wait, in order, and are formed into
 * rounds once the server is released (hold 0), e.g. to hand over a whole
 * wavefront's requests at once.  npm_drain releases a hold.               */
npm_status npm_server_hold(npm_server *srv, int32_t hold);
/* Blocks until the request has completed on the device (timeout_us < 0:
 * no limit; NPM_ERR_TIMEOUT on expiry; NPM_ERR_STATE without a limit while
 * the server is held and the request is not yet in a round).               */
npm_status npm_wait(npm_server *srv, uint64_t req, int64_t timeout_us);
/* Blocks until every submitted request has completed.                       */
npm_status npm_drain(npm_server *srv);
/* Timestamps of a completed request.                                       */
npm_status npm_request_info_get(npm_server *srv, uint64_t req, npm_request_info *out);
npm_status npm_server_stats_get(npm_server *srv, npm_server_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* NPM_SERVE_H */
