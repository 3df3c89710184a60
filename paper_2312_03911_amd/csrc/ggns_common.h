// Internal structures shared by the engine's host code and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ggns.h"

namespace ggns {

// Stream tags of the counter-based generator (word 3 of the counter holds
// tag << 24 | sub).
enum : uint32_t { TAG_INIT = 1, TAG_START = 2, TAG_P0 = 3, TAG_EPS = 4, TAG_RES = 5 };

constexpr int kMaxD = 256;
constexpr int kMaxLive = 4096;
constexpr int kMaxComp = 8;
constexpr int kWalkThreads = 256;

// Read-only description of one run on the device: settings plus the byte
// offsets of its arrays in the arena.
struct RunDev {
    int32_t d, n_live, n_kill, kind, prec, n_comp;
    int32_t n_steps_max, min_ref, max_ref, prune_streak;
    int32_t term_kind, max_iter;
    int32_t C, G;              // walk tile: coordinates per lane, lanes per walker
    int32_t dp, var;           // padded dimension G*C; kernel variant (family / slots)
    int32_t nprm;              // elements of the converted parameter block
    int32_t nprm_bytes_lds;    // bytes staged to LDS by the walk (0: read from global)
    double lo, hi, dt_init, delta_p, out_hi, out_lo, dt_down, dt_up, term_tol;
    uint64_t seed;
    int64_t param_offset;
    int64_t off_acc, off_prm, off_prm_bf16, off_live_x, off_live_logl, off_killed, off_surv,
        off_start, off_walk_x, off_walk_logl, off_dead_logl, off_dead_logw;
    int64_t dead_cap;
    // per-run trace (parity tests); null when off
    void *trace_x;
    double *trace_logl;
    int32_t *trace_out;
    int32_t trace_steps, mw;   // mw: wavefronts per group of 16 walkers (matrix-core walk)
    int32_t noise_mode;        // 1: one noise normal per walker and step
    int32_t walk_mode;         // 1: the batch-minimum loop (first walk, then its continuation)
    int64_t off_wstate;        // walk_mode 1: walker states at the end of the first walk
    int64_t wstate_stride;     // bytes per walker of off_wstate
    // positions of the dead points (posterior samples), caller-owned; null when off
    void *dead_x;
    int64_t dead_x_cap;        // rows of dead_x
    // clusters (cluster_mode 1): labels per live slot, the cluster table, the
    // live slots grouped by cluster, k-nearest-neighbour lists, walker clusters
    int32_t cluster_mode, cluster_kmax;
    int64_t off_label, off_cltab, off_members, off_knn, off_start_cl;
    int64_t off_knn_d;         // the neighbours' squared distances (double) beside off_knn
    int64_t off_knn_part, off_knn_part_s;   // per query and share: partial neighbour lists
    int64_t off_surv_sorted;   // survivors of the last kill in (log L, slot) order
    int64_t off_fin;           // run summary: five FP64 partials per chunk of dead records
    int32_t fin_chunks, pad_fin;   // chunks of kFinChunk records covering dead_cap
};

constexpr int kFinThreads = 256;                      // run summary: threads per chunk
constexpr int kFinPerThread = 16;                     // records per thread
constexpr int kFinChunk = kFinThreads * kFinPerThread; // records per chunk (one workgroup)
constexpr int kClMax = 64;      // clusters per run
constexpr int kKnnMax = 32;     // neighbours kept per point (largest cluster_kmax)
constexpr int kKnnPass = 8;     // neighbours found per search pass
constexpr int kKnnPasses = kKnnMax / kKnnPass;
constexpr int kKnnSplit = 16;   // shares of the candidate range searched in parallel

// Per-run cluster table (arena).
struct ClusterTab {
    double clx[kClMax];         // log Xbar_p (-inf: removed)
    double cum[kClMax];         // spawning CDF over clusters with survivors (scaled)
    int32_t cn[kClMax];         // live points per cluster
    int32_t soff[kClMax + 1];   // survivors grouped by cluster: offsets into the survivor list
    int32_t moff[kClMax + 1];   // live slots grouped by cluster: offsets into members
    int32_t n_clusters, n_splits, stopping, pad;
    // neighbour search in passes of kKnnPass: clusters whose loop needs the
    // next pass, the run's search finished, loops cut at kKnnMax
    int32_t need[kClMax];
    int32_t cc_done, n_cut, pad2[2];
    // the cluster recursion's moments, as logarithms (Eqs. update0-update9,
    // new0-new6): Zbar_p, (Z_p^2)bar, (Z X_p)bar, (Z_p X_p)bar, (X_p^2)bar,
    // (X_p X_q)bar
    double lzp[kClMax], lz2p[kClMax], lzx[kClMax], lzpx[kClMax], lx2[kClMax];
    double lxx[kClMax * kClMax];
};

// Mutable per-run state on the device.
struct Acc {
    double log_z, log_x, log_z2, dt, lstar, log_xl_max, h, sigma_kl, sigma_mom;
    long long iter, evals, n_dead, steps_out, steps_in, prunes, nosave;
    unsigned long long it_outs, it_steps;
    int32_t state, summary_pending;
    int32_t n_clusters;            // cluster indices in use (cluster mode)
    int32_t order_ok;              // 1: killed[] and surv_sorted[] hold the last kill's order
    int32_t win_a, win_b;          // walk_mode 1: the saving window [win_a, win_b] of this walk
    unsigned long long replayed;   // walk_mode 1: steps walked again
};

// A walk work item: walkers [m_begin, m_end) of one run.
struct Tile {
    int32_t run, m_begin, m_end, pad;
};

template <typename T>
__host__ __device__ inline T *at(void *arena, int64_t off) {
    return reinterpret_cast<T *>(reinterpret_cast<char *>(arena) + off);
}

// Launchers (defined in the .hip files).
void launch_prepare(void *arena, const RunDev *runs_dev, int n_runs, const double *params,
                    hipStream_t s, int init_state);
int launch_init_class(void *arena, const RunDev *runs_dev, const Tile *tiles, int n_tiles, int prec,
                      int C, int kind, hipStream_t s);
void launch_evidence(void *arena, const RunDev *runs_dev, int n_runs, int final_sweep,
                     int any_cluster, hipStream_t s);
void launch_finalize(void *arena, const RunDev *runs_dev, int n_runs, int max_chunks, hipStream_t s);
void launch_replace(void *arena, const RunDev *runs_dev, int n_runs, int max_kd, hipStream_t s);
// phase 1: first walk of the batch-minimum loop (walk_mode 1 runs; others
// return at once); phase 2: its continuation, or the per-walker walk
int launch_walk_class(void *arena, const RunDev *runs_dev, const Tile *tiles, int n_tiles,
                      int prec, int C, int kind, int gf, size_t lds_bytes, int phase, hipStream_t s);
bool mfma_shape_ok(int d_pad, int waves);
int launch_walk_mfma(void *arena, const RunDev *runs_dev, const Tile *tiles, int n_tiles,
                     int d_pad, int waves, int nz, int phase, hipStream_t s);
// bytes of one walker's saved state between the two walk launches
int64_t walker_state_bytes(int d_pad, int elem_bytes);
int launch_loglike(void *arena, const RunDev *run_dev, const RunDev &run_host, const void *x,
                   int64_t n, double *logl, void *grad, const double *gout, hipStream_t s);
int64_t plain_workspace_bytes(const RunDev &R);
int launch_ext_begin(void *arena, const RunDev *runs_dev, int run, const RunDev &R, void *ws,
                     hipStream_t s);
int launch_ext_step(void *arena, const RunDev *runs_dev, int run, const RunDev &R, void *ws, int t,
                    hipStream_t s);
void ext_buffers(const RunDev &R, void *ws, double **x, double **logl, double **grad,
                 int32_t **active);
int launch_walk_plain(void *arena, const RunDev *runs_dev, int run, const RunDev &R, void *ws,
                      int poll_every, hipStream_t s);
int launch_noise_normals(uint64_t seed, int iteration, int n_walkers, int n_blocks, int steps,
                         float *normals, uint32_t *words, float *checksum, hipStream_t s);
int launch_gather_acc(void *arena, const RunDev *runs_dev, int n_runs, ggns_run_stats *mirror,
                      hipStream_t s);
int launch_clusters(void *arena, const RunDev *runs_dev, int n_runs, int max_live, int final_sweep,
                    bool any_fp64, bool any_fp32, hipStream_t s);
void launch_set_vars(void *arena, const RunDev *run_dev, double log_z, double log_x, double dt,
                     long long iter, hipStream_t s);

}  // namespace ggns
