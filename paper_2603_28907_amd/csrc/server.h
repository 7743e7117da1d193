// server.h -- the serving loop behind mc_server_* (included at the end of
// api.hip, which provides the problem handle and the batched MCMC step).
//
// One scheduler thread per server:
//
//   loop:
//     launch one round (k steps of every resident job, one graph per
//       surface count) on the server stream                       [async]
//     admit queue heads while slots and memory allow; set them up:
//       handle, uploads, chains from the shared start, initial log
//       posterior (enqueued behind the round)                     [overlaps]
//     wait for the round; jobs that reached n_steps get their summary
//       computed on the device, copied to the host, and their device
//       memory freed; admitted jobs become resident
//
// Jobs join and leave only at round boundaries, so a job's Philox counters
// (seed, step) and its launch shape never depend on what else is resident.
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

#include "summary.h"

namespace {

struct ServerJob {
    int64_t id = 0;
    // copy of the description
    int S = 0, R = 0, C = 0, n_s = 0, n_pix = 0, n = 0, block = 0, rpt = 0;
    double X = 0, Y = 0, atten = 0, step = 0;
    std::vector<double> density, top, car_r, pos, dirs, expo, init;
    std::vector<int32_t> counts;
    int64_t n_steps = 0;
    uint64_t seed = 0;
    double r_step = 0;   // > 0: every chain samples its r (logit-scale random walk of this step)
    size_t footprint = 0;
    // progress
    int status = MC_JOB_QUEUED;
    int64_t steps_done = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    // device state while resident
    mc_problem *p = nullptr;
    void *H = nullptr;
    double *lp = nullptr, *dsum = nullptr, *r = nullptr;
    int64_t *acc = nullptr, *acc_r = nullptr;
    // summary
    std::vector<double> mean, sd, map_state, r_mean;
    double accept_rate = 0, map_lp = 0, r_accept_rate = 0;
    int map_chain = 0;
    std::string err;
};

size_t round_up(size_t b) { return (b + 4095) & ~(size_t)4095; }

// Device bytes a job holds while resident: chain state and the MCMC
// workspaces, geometry and per-ray tables, summary buffer; each allocation
// rounded to 4 KB, plus a fixed allowance for the handle's small buffers.
size_t job_footprint(const ServerJob &j, int prec) {
    const size_t sz = prec == MC_F64 ? 8 : 4;
    const size_t N = (size_t)j.R * j.C, M = (size_t)(j.S - 1) * N, nr = (size_t)j.n_s * j.n_pix;
    mc_tuning t = default_tuning(prec, N);
    if (j.block > 0) t.block = j.block;
    if (j.rpt > 0) t.rays_per_thread = j.rpt;
    const size_t rpb = (size_t)t.block * t.rays_per_thread;
    const size_t tiles = nr ? (nr + rpb - 1) / rpb : 0;
    size_t b = 0;
    b += 2 * round_up((size_t)j.n * M * sz);                 // states, proposals
    b += 3 * round_up((size_t)j.n * 8);                      // lp, lp scratch, acceptances
    b += round_up((size_t)j.n * tiles * 8);                  // likelihood partials
    b += round_up(N * sz) + round_up(N * 8);                 // top surface
    b += round_up((size_t)j.n_s * 3 * sz);                   // sensors
    b += 9 * round_up(nr * sz) + 2 * round_up(nr * 8);       // directions, ray constants, exposure, count terms
    b += round_up((3 * M + 4) * 8);                          // summary / start state
    if (j.r_step > 0) b += 4 * round_up((size_t)j.n * (j.S - 1) * 8);   // r, r acceptances, w-statistics
    return b + (64u << 10);
}

}  // namespace

struct mc_server {
    mc_server_config cfg{};
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv, idle_cv;
    std::deque<ServerJob *> queue;
    std::vector<ServerJob *> resident;
    std::map<int64_t, ServerJob *> jobs;
    int64_t next_id = 1;
    bool stop = false, drain = true;
    std::thread th;
    hipStream_t st = nullptr;
    std::chrono::steady_clock::time_point t0;
    mc_server_stats stats{};
    std::string err;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

std::string g_server_error;

mc_status server_fail(mc_server *s, mc_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    else g_server_error = buf;
    return code;
}

void release_device(ServerJob *j) {
    if (j->p) mc_destroy(j->p);
    j->p = nullptr;
    for (void *q : {j->H, (void *)j->lp, (void *)j->dsum, (void *)j->acc, (void *)j->r, (void *)j->acc_r})
        if (q) (void)hipFree(q);
    j->H = nullptr;
    j->lp = nullptr;
    j->dsum = nullptr;
    j->acc = nullptr;
    j->r = nullptr;
    j->acc_r = nullptr;
}

// Handle, uploads, chain start and initial log posterior of an admitted job
// (device work enqueued on the server stream).
mc_status setup_job(mc_server *s, ServerJob *j) {
    mc_problem *p = nullptr;
    mc_status r = mc_create(s->cfg.device, s->cfg.precision, &p);
    if (r != MC_OK) {
        j->err = g_create_error;
        return r;
    }
    j->p = p;
    auto check = [&](mc_status code) {
        if (code != MC_OK) j->err = p->err;
        return code;
    };
    if ((r = check(load_geometry_grid(p, j->S, j->R, j->C, j->X, j->Y, j->density.data(), j->top.data(),
                                      j->car_r.data()))) != MC_OK)
        return r;
    if ((r = check(set_sensors(p, j->n_s, j->pos.data(), j->n_pix, j->dirs.data(), j->expo.data(), j->atten))) !=
        MC_OK)
        return r;
    if (j->n_s * j->n_pix > 0 && (r = check(set_counts(p, j->counts.data()))) != MC_OK) return r;
    if (j->block > 0 || j->rpt > 0) {
        mc_tuning t = p->tune;
        if (j->block > 0) t.block = j->block;
        if (j->rpt > 0) t.rays_per_thread = j->rpt;
        if ((r = check(mc_set_tuning(p, &t))) != MC_OK) return r;
    }
    const size_t M = (size_t)(j->S - 1) * j->R * j->C, sz = elem_size(p);
    DeviceGuard g(s->cfg.device);
    if (hipMalloc(&j->H, (size_t)j->n * M * sz) != hipSuccess || hipMalloc((void **)&j->lp, 8 * (size_t)j->n) != hipSuccess ||
        hipMalloc((void **)&j->acc, 8 * (size_t)j->n) != hipSuccess ||
        hipMalloc((void **)&j->dsum, 8 * (3 * M + 4)) != hipSuccess) {
        j->err = "device allocation failed";
        return MC_ERR_NOMEM;
    }
    if (hipMemcpy(j->dsum, j->init.data(), 8 * M, hipMemcpyHostToDevice) != hipSuccess) {
        j->err = "upload of the start state failed";
        return MC_ERR_DEVICE;
    }
    if (j->r_step > 0) {
        // every chain starts at the job's r
        const size_t nr = (size_t)j->n * (j->S - 1);
        std::vector<double> r0(nr);
        for (size_t i = 0; i < nr; ++i) r0[i] = j->car_r[i % (j->S - 1)];
        if (hipMalloc((void **)&j->r, 8 * nr) != hipSuccess || hipMalloc((void **)&j->acc_r, 8 * nr) != hipSuccess) {
            j->err = "device allocation failed";
            return MC_ERR_NOMEM;
        }
        if (hipMemcpy(j->r, r0.data(), 8 * nr, hipMemcpyHostToDevice) != hipSuccess) {
            j->err = "upload of the r start failed";
            return MC_ERR_DEVICE;
        }
        hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s->st,
                           (unsigned long long *)j->acc_r, nr);
    }
    const size_t tot = (size_t)j->n * M;
    const unsigned gb = (unsigned)std::min<size_t>((tot + 255) / 256, 65535);
    if (s->cfg.precision == MC_F64)
        hipLaunchKernelGGL(k_broadcast_init<double>, dim3(gb), dim3(256), 0, s->st, j->dsum, (double *)j->H, j->n, (int)M);
    else
        hipLaunchKernelGGL(k_broadcast_init<float>, dim3(gb), dim3(256), 0, s->st, j->dsum, (float *)j->H, j->n, (int)M);
    hipLaunchKernelGGL(k_fill_u64, dim3((j->n + 255) / 256), dim3(256), 0, s->st, (unsigned long long *)j->acc,
                       (size_t)j->n);
    if (hipGetLastError() != hipSuccess) {
        j->err = "launch failed";
        return MC_ERR_DEVICE;
    }
    if ((r = check(logpost_batch(p, j->n, j->H, j->lp, nullptr, s->st))) != MC_OK) return r;
    return MC_OK;
}

// k steps of every job in `group` (one surface count).
template <typename T, int S>
mc_status run_group(mc_server *s, const std::vector<ServerJob *> &group, int k) {
    const int np = (int)group.size();
    std::vector<mc_problem *> ps(np);
    std::vector<mc_run_config> cfgs(np);
    std::vector<int> nch(np);
    std::vector<void *> hs(np);
    std::vector<double *> lps(np);
    std::vector<int64_t *> accs(np);
    for (int i = 0; i < np; ++i) {
        ServerJob *j = group[i];
        ps[i] = j->p;
        cfgs[i] = mc_run_config{0, k, k, j->step, nullptr, j->seed, (uint64_t)j->steps_done};
        if (j->r_step > 0) {
            cfgs[i].r_state = j->r;
            cfgs[i].r_step = j->r_step;
            cfgs[i].n_accept_r = j->acc_r;
        }
        nch[i] = j->n;
        hs[i] = j->H;
        lps[i] = j->lp;
        accs[i] = j->acc;
    }
    std::lock_guard<std::mutex> lock(g_multi_mu);
    return mcmc_multi_impl<T, S>(np, ps.data(), cfgs.data(), nch.data(), hs.data(), lps.data(), accs.data(), s->st,
                                 false);
}

mc_status run_round(mc_server *s, const std::vector<ServerJob *> &res, int k) {
    // one group per surface count and per kind of r (fixed or sampled)
    for (int gi = 0; gi < 2 * (kMaxSurfaces - 1); ++gi) {
        const int S = 2 + gi / 2;
        const bool hier = gi % 2 == 1;
        std::vector<ServerJob *> group;
        for (ServerJob *j : res)
            if (j->S == S && (j->r_step > 0) == hier) group.push_back(j);
        if (group.empty()) continue;
        mc_status r;
        if (s->cfg.precision == MC_F64) {
            r = S == 2 ? run_group<double, 2>(s, group, k) : S == 3 ? run_group<double, 3>(s, group, k)
                                                                      : run_group<double, 4>(s, group, k);
        } else {
            r = S == 2 ? run_group<float, 2>(s, group, k) : S == 3 ? run_group<float, 3>(s, group, k)
                                                                     : run_group<float, 4>(s, group, k);
        }
        if (r != MC_OK) {
            for (ServerJob *j : group) j->err = group[0]->p->err;
            return r;
        }
    }
    return MC_OK;
}

// Summary kernels of a finished job (device), enqueued on the server stream.
void enqueue_summary(mc_server *s, ServerJob *j) {
    const int M = (j->S - 1) * j->R * j->C;
    const dim3 gm((M + 255) / 256);
    double *out = j->dsum;
    if (s->cfg.precision == MC_F64)
        hipLaunchKernelGGL(k_node_summary<double>, gm, dim3(256), 0, s->st, (const double *)j->H, j->n, M, out, out + M);
    else
        hipLaunchKernelGGL(k_node_summary<float>, gm, dim3(256), 0, s->st, (const float *)j->H, j->n, M, out, out + M);
    hipLaunchKernelGGL(k_chain_summary<256>, dim3(1), dim3(256), 0, s->st, (const double *)j->lp,
                       (const int64_t *)j->acc, j->n, out + 3 * M);
    if (s->cfg.precision == MC_F64)
        hipLaunchKernelGGL(k_copy_chain<double>, gm, dim3(256), 0, s->st, (const double *)j->H, M,
                           (const double *)(out + 3 * M + 1), out + 2 * M);
    else
        hipLaunchKernelGGL(k_copy_chain<float>, gm, dim3(256), 0, s->st, (const float *)j->H, M,
                           (const double *)(out + 3 * M + 1), out + 2 * M);
}

void mark_failed(mc_server *s, ServerJob *j, const std::string &why) {
    release_device(j);
    std::lock_guard<std::mutex> lock(s->mu);
    j->status = MC_JOB_FAILED;
    if (j->err.empty()) j->err = why;
    j->t_done = s->now();
    s->stats.failed += 1;
    s->stats.bytes_in_use -= j->footprint;
    s->idle_cv.notify_all();
}

void scheduler(mc_server *s) {
    (void)hipSetDevice(s->cfg.device);
    std::vector<ServerJob *> resident;
    for (;;) {
        // 1. launch a round over the resident jobs
        int k = 0;
        double t_round = s->now();
        mc_status rr = MC_OK;
        if (!resident.empty()) {
            int64_t left = INT64_MAX;
            for (ServerJob *j : resident) left = std::min(left, j->n_steps - j->steps_done);
            k = (int)std::min<int64_t>(left, s->cfg.steps_per_round);
            rr = run_round(s, resident, k);
        }
        // 2. admission, overlapping the round
        std::vector<ServerJob *> admitted;
        {
            std::unique_lock<std::mutex> lock(s->mu);
            for (;;) {
                if (s->stop && (!s->drain || (s->queue.empty() && resident.empty()))) break;
                while (!s->queue.empty()) {
                    ServerJob *h = s->queue.front();
                    if ((int)(resident.size() + admitted.size()) >= s->cfg.max_jobs) break;
                    if (s->stats.bytes_in_use + h->footprint > s->budget) break;
                    s->queue.pop_front();
                    h->status = MC_JOB_RUNNING;
                    h->t_admit = s->now();
                    s->stats.bytes_in_use += h->footprint;
                    s->stats.peak_bytes = std::max(s->stats.peak_bytes, s->stats.bytes_in_use);
                    s->stats.admitted += 1;
                    admitted.push_back(h);
                }
                if (!admitted.empty() || !resident.empty()) break;
                s->cv.wait_for(lock, std::chrono::milliseconds(20));
            }
            if (s->stop && (!s->drain || (s->queue.empty() && resident.empty() && admitted.empty()))) {
                lock.unlock();
                (void)hipStreamSynchronize(s->st);
                break;
            }
        }
        std::vector<ServerJob *> ready;
        for (ServerJob *j : admitted) {
            if (setup_job(s, j) == MC_OK) ready.push_back(j);
            else mark_failed(s, j, "set-up failed");
        }
        // 3. wait for the round, then retire finished jobs
        hipError_t se = hipStreamSynchronize(s->st);
        if (!resident.empty()) {
            const double t_end = s->now();
            std::vector<ServerJob *> keep, finished;
            if (rr != MC_OK || se != hipSuccess) {
                for (ServerJob *j : resident)
                    mark_failed(s, j, se != hipSuccess ? hipGetErrorString(se) : "round failed");
            } else {
                for (ServerJob *j : resident) {
                    j->steps_done += k;
                    (j->steps_done >= j->n_steps ? finished : keep).push_back(j);
                }
                for (ServerJob *j : finished) enqueue_summary(s, j);
                std::vector<std::vector<double>> host(finished.size()), hr(finished.size());
                std::vector<std::vector<int64_t>> hacc(finished.size());
                for (size_t i = 0; i < finished.size(); ++i) {
                    ServerJob *j = finished[i];
                    const size_t M = (size_t)(j->S - 1) * j->R * j->C;
                    host[i].resize(3 * M + 3);
                    (void)hipMemcpyAsync(host[i].data(), j->dsum, 8 * (3 * M + 3), hipMemcpyDeviceToHost, s->st);
                    if (j->r) {
                        hr[i].resize((size_t)j->n * (j->S - 1));
                        hacc[i].resize(hr[i].size());
                        (void)hipMemcpyAsync(hr[i].data(), j->r, 8 * hr[i].size(), hipMemcpyDeviceToHost, s->st);
                        (void)hipMemcpyAsync(hacc[i].data(), j->acc_r, 8 * hacc[i].size(), hipMemcpyDeviceToHost,
                                             s->st);
                    }
                }
                se = hipStreamSynchronize(s->st);
                for (size_t i = 0; i < finished.size(); ++i) {
                    ServerJob *j = finished[i];
                    if (se != hipSuccess) {
                        mark_failed(s, j, hipGetErrorString(se));
                        continue;
                    }
                    const size_t M = (size_t)(j->S - 1) * j->R * j->C;
                    release_device(j);
                    std::lock_guard<std::mutex> lock(s->mu);
                    j->mean.assign(host[i].begin(), host[i].begin() + M);
                    j->sd.assign(host[i].begin() + M, host[i].begin() + 2 * M);
                    j->map_state.assign(host[i].begin() + 2 * M, host[i].begin() + 3 * M);
                    j->map_lp = host[i][3 * M];
                    j->map_chain = (int)host[i][3 * M + 1];
                    j->accept_rate = host[i][3 * M + 2] / ((double)j->n * (double)j->n_steps);
                    if (!hr[i].empty()) {
                        // mean r of every free surface over the chains' last states, in chain order
                        const int S1 = j->S - 1;
                        j->r_mean.assign(S1, 0.0);
                        double na = 0.0;
                        for (int c = 0; c < j->n; ++c)
                            for (int l = 0; l < S1; ++l) {
                                j->r_mean[l] += hr[i][(size_t)c * S1 + l] / j->n;
                                na += (double)hacc[i][(size_t)c * S1 + l];
                            }
                        j->r_accept_rate = na / ((double)j->n * S1 * (double)j->n_steps);
                    }
                    j->status = MC_JOB_DONE;
                    j->t_done = s->now();
                    s->stats.done += 1;
                    s->stats.bytes_in_use -= j->footprint;
                }
            }
            resident.swap(keep);
            std::lock_guard<std::mutex> lock(s->mu);
            s->stats.rounds += 1;
            s->stats.busy_seconds += t_end - t_round;
            s->idle_cv.notify_all();
        }
        for (ServerJob *j : ready) resident.push_back(j);
        {
            std::lock_guard<std::mutex> lock(s->mu);
            s->resident = resident;
            s->stats.max_resident = std::max(s->stats.max_resident, (int)resident.size());
        }
    }
    // abandoned jobs (destroy without drain)
    for (ServerJob *j : resident) mark_failed(s, j, "server stopped");
}

}  // namespace

extern "C" {

mc_status mc_server_create(const mc_server_config *cfg, mc_server **out) {
    if (!out || !cfg) return server_fail(nullptr, MC_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (cfg->precision != MC_F32 && cfg->precision != MC_F64)
        return server_fail(nullptr, MC_ERR_ARG, "precision %d", cfg->precision);
    if (cfg->max_jobs < 1 || cfg->steps_per_round < 1)
        return server_fail(nullptr, MC_ERR_ARG, "max_jobs and steps_per_round must be >= 1");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return server_fail(nullptr, MC_ERR_DEVICE, "no HIP device");
    if (cfg->device < 0 || cfg->device >= count) return server_fail(nullptr, MC_ERR_ARG, "device %d", cfg->device);
    mc_server *s = new mc_server();
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    DeviceGuard g(cfg->device);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        delete s;
        return server_fail(nullptr, MC_ERR_DEVICE, "hipMemGetInfo failed");
    }
    s->budget = cfg->memory_budget ? cfg->memory_budget : (free_b > cfg->reserve ? free_b - cfg->reserve : 0);
    s->stats.budget = s->budget;
    if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return server_fail(nullptr, MC_ERR_DEVICE, "stream creation failed");
    }
    s->th = std::thread(scheduler, s);
    *out = s;
    return MC_OK;
}

void mc_server_destroy(mc_server *s, int drain) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->drain = drain != 0;
        if (!s->drain) {
            for (ServerJob *j : s->queue) {
                j->status = MC_JOB_FAILED;
                j->err = "server stopped";
            }
            s->queue.clear();
        }
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    {
        DeviceGuard g(s->cfg.device);
        for (auto &kv : s->jobs) {
            release_device(kv.second);
            delete kv.second;
        }
        if (s->st) (void)hipStreamDestroy(s->st);
    }
    delete s;
}

const char *mc_server_last_error(const mc_server *s) { return s ? s->err.c_str() : g_server_error.c_str(); }

mc_status mc_server_submit(mc_server *s, const mc_job_desc *d, int64_t *job_id) {
    if (!s || !d || !job_id) return server_fail(s, MC_ERR_ARG, "NULL argument");
    const int S = d->n_surfaces, R = d->n_rows, C = d->n_cols;
    if (S < 2 || S > kMaxSurfaces || R < 3 || C < 3 || (long long)R * C > kMaxNodes)
        return server_fail(s, MC_ERR_ARG, "grid %d surfaces %dx%d not supported", S, R, C);
    if (d->n_sensors < 0 || d->n_pix < 0 || (d->n_sensors > 0 && d->n_pix == 0))
        return server_fail(s, MC_ERR_ARG, "sensor sizes");
    if (d->n_chains <= 0 || d->n_chains > 65535) return server_fail(s, MC_ERR_ARG, "n_chains %d", d->n_chains);
    if (d->n_steps < 1 || d->n_steps >= (1LL << 47)) return server_fail(s, MC_ERR_ARG, "n_steps");
    if (!(d->step_size >= 0) || !std::isfinite(d->step_size)) return server_fail(s, MC_ERR_ARG, "step_size");
    if (!(d->r_step >= 0) || !std::isfinite(d->r_step)) return server_fail(s, MC_ERR_ARG, "r_step");
    if (!d->density || !d->top || !d->car_r || !d->init) return server_fail(s, MC_ERR_ARG, "NULL array");
    const size_t nr = (size_t)d->n_sensors * d->n_pix, N = (size_t)R * C;
    if (nr > 0 && (!d->sensor_pos || !d->dirs || !d->exposure || !d->counts))
        return server_fail(s, MC_ERR_ARG, "NULL sensor array");
    ServerJob *j = new ServerJob();
    j->S = S;
    j->R = R;
    j->C = C;
    j->X = d->extent_x;
    j->Y = d->extent_y;
    j->density.assign(d->density, d->density + S);
    j->top.assign(d->top, d->top + N);
    j->car_r.assign(d->car_r, d->car_r + S - 1);
    j->n_s = d->n_sensors;
    j->n_pix = d->n_pix;
    if (d->n_sensors > 0) {
        j->pos.assign(d->sensor_pos, d->sensor_pos + 3 * (size_t)d->n_sensors);
        j->dirs.assign(d->dirs, d->dirs + 3 * nr);
        j->expo.assign(d->exposure, d->exposure + nr);
        j->counts.assign(d->counts, d->counts + nr);
    }
    j->atten = d->atten_len;
    j->n = d->n_chains;
    j->init.assign(d->init, d->init + (size_t)(S - 1) * N);
    j->n_steps = d->n_steps;
    j->step = d->step_size;
    j->seed = d->seed;
    j->block = d->block;
    j->rpt = d->rays_per_thread;
    j->r_step = d->r_step;
    j->footprint = job_footprint(*j, s->cfg.precision);
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) {
        delete j;
        return server_fail(s, MC_ERR_STATE, "server is stopping");
    }
    if (j->footprint > s->budget) {
        const size_t need = j->footprint;
        delete j;
        return server_fail(s, MC_ERR_NOMEM, "job needs %zu bytes, budget is %zu", need, s->budget);
    }
    j->id = s->next_id++;
    j->t_submit = s->now();
    s->jobs[j->id] = j;
    s->queue.push_back(j);
    s->stats.submitted += 1;
    *job_id = j->id;
    s->cv.notify_all();
    return MC_OK;
}

mc_status mc_server_poll(mc_server *s, int64_t job_id, mc_job_info *info, double *mean, double *sd,
                         double *map_state) {
    if (!s || !info) return server_fail(s, MC_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return server_fail(s, MC_ERR_ARG, "unknown job %lld", (long long)job_id);
    const ServerJob *j = it->second;
    info->status = j->status;
    info->map_chain = j->map_chain;
    info->steps_done = j->steps_done;
    info->t_submit = j->t_submit;
    info->t_admit = j->t_admit;
    info->t_done = j->t_done;
    info->accept_rate = j->accept_rate;
    info->map_logpost = j->map_lp;
    info->footprint = j->footprint;
    for (int l = 0; l < 3; ++l) info->r_mean[l] = l < (int)j->r_mean.size() ? j->r_mean[l] : 0.0;
    info->r_accept_rate = j->r_accept_rate;
    if (j->status == MC_JOB_DONE) {
        if (mean) std::copy(j->mean.begin(), j->mean.end(), mean);
        if (sd) std::copy(j->sd.begin(), j->sd.end(), sd);
        if (map_state) std::copy(j->map_state.begin(), j->map_state.end(), map_state);
    }
    if (j->status == MC_JOB_FAILED) s->err = j->err;
    return MC_OK;
}

mc_status mc_server_release(mc_server *s, int64_t job_id) {
    if (!s) return MC_ERR_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return server_fail(s, MC_ERR_ARG, "unknown job %lld", (long long)job_id);
    if (it->second->status != MC_JOB_DONE && it->second->status != MC_JOB_FAILED)
        return server_fail(s, MC_ERR_STATE, "job %lld has not finished", (long long)job_id);
    delete it->second;
    s->jobs.erase(it);
    return MC_OK;
}

mc_status mc_server_wait_idle(mc_server *s, double timeout_s) {
    if (!s) return MC_ERR_ARG;
    std::unique_lock<std::mutex> lock(s->mu);
    const bool ok = s->idle_cv.wait_for(lock, std::chrono::duration<double>(timeout_s), [&] {
        return s->stats.done + s->stats.failed >= s->stats.submitted;
    });
    return ok ? MC_OK : server_fail(s, MC_ERR_STATE, "time-out with %lld jobs unfinished",
                                    (long long)(s->stats.submitted - s->stats.done - s->stats.failed));
}

mc_status mc_server_get_stats(mc_server *s, mc_server_stats *st) {
    if (!s || !st) return MC_ERR_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    *st = s->stats;
    st->resident = (int)s->resident.size();
    st->queued = (int)s->queue.size();
    st->now = s->now();
    return MC_OK;
}

}  // extern "C"
