// Host side of the kernels: the launch helper that times a dispatch with
// an event pair bound to it, and the launchers each .hip file defines.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "sf_dev.h"

// Timing of the next launch: when the handle profiles its kernels it puts
// an event pair here, and the next sf_launch hands it to the dispatch
// itself (hipExtLaunchKernelGGL), so that the recorded interval is the
// kernel's execution without the gaps of separately enqueued event
// markers.  One launch consumes the pair.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents g_launch_ev;

template <typename... KArgs, typename... Args>
inline void sf_launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t shm, hipStream_t s, Args... args) {
    const LaunchEvents ev = g_launch_ev;
    g_launch_ev = LaunchEvents{};
    if (ev.start)
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shm, s, ev.start, ev.stop, 0u, KArgs(args)...);
    else
        hipLaunchKernelGGL(kernel, grid, block, shm, s, KArgs(args)...);
}

// kernel launchers (defined in the .hip files)
void launch_weather_mu(const float *mu_class, const float *film, const uint8_t *pav, int W, int S,
                       float *mu_out, hipStream_t st);
void launch_quantise_roads(const float2 *xy, int2 *q, int P, hipStream_t st);
void launch_prep_tris(const float *verts, const uint8_t *surf, float4 *tri, int T, hipStream_t st);
void launch_tri_friction(const float *scale, float4 *tri, int T, hipStream_t st);
void launch_world_bbox(const int *roff, const float2 *xy, const int *toff, const float *verts, int W,
                       float4 *bbox, hipStream_t st);
void launch_grid_count(const DevWorld &Wd, const float *verts, int T, int P, int *tri_cnt,
                       int *pt_cnt, hipStream_t st);
void launch_grid_fill(const DevWorld &Wd, const float *verts, int T, int P, int *tri_cursor,
                      int *pt_cursor, int *tri_items, int *pt_items, hipStream_t st);
void launch_grid_finish(const DevWorld &Wd, int CT, int CP, int *tri_items, int *pt_items,
                        float4 *tri_rec, int4 *pt_cell, int *pt_occ, int *tri_work, int *pt_work,
                        hipStream_t st);
void launch_scan(const int *in, int *out, int n, int *tmp, hipStream_t st);  // exclusive, out[n]
void launch_world_of(const int *aoff, int W, int *world_of, hipStream_t st);
void launch_agent_desc(const int *aoff, const int *roff, const GridHdr *grid, int W, int4 *agent_world,
                       GridHdr *agent_grid, hipStream_t st);
void launch_reset(const DevParams &P, const DevWorld &Wd, float *st, int *ist, const uint8_t *mask,
                  int bump_episode, hipStream_t s);
void launch_step(const DevParams &P, const DevWorld &Wd, const DevSur &Su, bool use_sur, float *st, int *ist,
                 const float *act, float h, int S, float *reward, uint8_t *done, uint8_t *events, uint32_t *rec,
                 int *rec_cnt, int rec_cap, const int4 *items, int block, int grid, int *queue, hipStream_t s);
void launch_step_bicycle(const DevParams &P, const DevWorld &Wd, float *st, int *ist, const float *act, float dt,
                         float *reward, uint8_t *done, uint8_t *events, uint32_t *rec, int *rec_cnt, int rec_cap,
                         const int4 *items, hipStream_t s);
void launch_obs_full(const DevParams &P, const DevWorld &Wd, const float *st, const int *ist, const float *film,
                     const uint8_t *pav, float *obs, int *counts, hipStream_t s);
void launch_ac_pack(const float *Pf, uint16_t *Wb, hipStream_t s);
void launch_actor_critic_save(const float *obs, const int *counts, const int *rows, int M, const float *Pf,
                              const uint16_t *Wb, float *mean, float *value, float *save, hipStream_t s);
void launch_actor_critic(const float *obs, const int *counts, int N, const float *Pf, const uint16_t *Wb,
                         float *mean, float *value, float *act, float steer_max, hipStream_t s);
void launch_sur_reduce(const float *grad, int tiles, float *out, hipStream_t s);
void launch_sur_grad_seq(const float *data, int M, const float *P, const uint16_t *Wb, float *grad, float *loss,
                         hipStream_t s);
void launch_obs(const DevParams &P, const DevWorld &Wd, const float *st, const int *ist, float *obs,
                int *dbg_idx, float4 *hint, int waves, hipStream_t s);
void launch_hint_clear(float4 *hint, int n, hipStream_t s);
void launch_obs_policy(const DevParams &P, const DevWorld &Wd, const float *st, const int *ist, float *obs,
                       float4 *hint, const uint16_t *W1, const float *b1, const uint16_t *W2, const float *b2,
                       const uint16_t *W3, const float *b3, float steer_max, float *act, hipStream_t s);
void launch_to_bf16(const float *src, uint16_t *dst, int n, hipStream_t s);
void launch_policy(const float *obs, int N, const uint16_t *W1, const float *b1, const uint16_t *W2,
                   const float *b2, const uint16_t *W3, const float *b3, float steer_max, float *act,
                   int tm, hipStream_t s);
void launch_sur_collect(const float *log, int n, int *flag, int *pos, int *scan_tmp, float *out, int max_out,
                        hipStream_t s);
void launch_sur_envelope(const float *x, int M, float *part, float *lo, float *hi, hipStream_t s);
void launch_sur_init(float *P, unsigned long long seed, hipStream_t s);
void launch_sur_pack(const float *P, uint16_t *Wb, hipStream_t s);
void launch_sur_grad(const float *data, int M, const float *P, const uint16_t *Wb, unsigned long long seed,
                     int tiles, float *grad, float *loss, hipStream_t s);
void launch_sur_eval(const float *data, int M, const float *P, const uint16_t *Wb, float *pred, hipStream_t s);
void launch_sur_adam(float *P, float *m, float *v, const float *grad, int tiles, float lr, float b1, float b2,
                     float eps, float c1, float c2, uint16_t *Wb, hipStream_t s);
void launch_sur_errors(const float *data, int M, const float *pred, float *err, hipStream_t s);
void launch_debug_raycast(const DevParams &P, const DevWorld &Wd, const float *st, float *out,
                          hipStream_t s);
void launch_touch_count(const unsigned *bits, const long long *off_host, unsigned long long *acc,
                        hipStream_t s);
void launch_ppo_sample(const float *mean, const float *Pf, const float *eps, int N, float *u, float *logp, float *mu,
                       float *act, float steer_max, hipStream_t s);
void launch_ppo_advantages(const float *rew, const uint8_t *done, const float *val, int T, int N, float gamma,
                           float lam, float *adv, float *ret, double *part, hipStream_t s);
int ppo_moment_blocks(long long n);
void launch_ppo_loss(const int *rows, int B, const float *mean_new, const float *val_new, const float *u,
                     const float *logp_old, const float *mu_old, const float *adv, const float *ret, const float *Pf,
                     const float *ls_old, float clip, float c_v, float *dout, float *part, double *stats,
                     hipStream_t s);
void launch_ppo_backward(const float *obs, const int *rows, int B, const float *save, const float *dout,
                         const float *Pf, const uint16_t *Wb, float *part, hipStream_t s);
int ppo_tiles(int B);
void launch_ppo_reduce(const float *part, int tiles, float *gpart, const double *stats, float c_e, float *grad,
                       double *sq, hipStream_t s);
int ppo_reduce_groups();
void launch_ppo_adam(float *P, float *m, float *v, const float *grad, const double *sq, float max_norm, float lr,
                     float b1, float b2, float eps, float c1, float c2, float *norm_out, hipStream_t s);
void launch_ppo_check_rows(const int *rows, long long n, int limit, int *flag, hipStream_t s);
