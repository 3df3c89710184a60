// Host side of the C ABI (include/ggns.h): validation, arena layout, walk
// tiling, and the launches behind each entry point.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ggns_device.h"

using namespace ggns;

namespace {

constexpr int64_t kAlign = 256;

// The fixed device buffer of ggns_hss_walk_plain_static.  In host code this
// name stands for the device symbol only: its device address (one per GPU)
// comes from hipGetSymbolAddress, taken once per device at context set-up.
__device__ __align__(256) unsigned char scratch[GGNS_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, resolved on first use (with the
// device current); nullptr if the runtime cannot give it.
void *scratch_for_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

bool valid_desc(const ggns_run_desc &r) {
    if (r.d < 1 || r.d > kMaxD) return false;
    if (r.n_live < 2 || r.n_live > kMaxLive) return false;
    if (r.n_kill < 1 || r.n_kill >= r.n_live) return false;
    if (r.lik_kind < 0 || r.lik_kind > GGNS_LIK_TORUS) return false;
    if (r.precision < 0 || r.precision > 2) return false;
    if ((r.lik_kind == GGNS_LIK_SHELLS || r.lik_kind == GGNS_LIK_GMM_DIAG) &&
        (r.n_comp < 1 || r.n_comp > kMaxComp))
        return false;
    if (!(r.prior_hi > r.prior_lo)) return false;
    if (!(r.dt_init > 0.0)) return false;
    if (r.n_steps_max < 1 || r.min_ref < 0 || r.max_ref < 0 || r.prune_streak < 0) return false;
    if (r.term_kind < GGNS_TERM_REMAINING_Z || r.term_kind > GGNS_TERM_XL_PEAK_DEAD) return false;
    if (!(r.term_tol > 0.0) || r.max_iter < 0) return false;
    if (r.param_offset < 0) return false;
    if (r.tile_c < 0 || r.tile_c > 16) return false;
    if (r.noise_mode != 0 && r.noise_mode != 1) return false;
    if (r.cluster_mode != 0 && r.cluster_mode != 1) return false;
    if (r.cluster_mode && (r.cluster_kmax < 2 || r.cluster_kmax > kKnnMax)) return false;
    if (r.walk_mode != 0 && r.walk_mode != 1) return false;
    // the batch-minimum loop needs a reflection count to stop on, and its
    // saving window starts no later than its end
    if (r.walk_mode == 1 && (r.max_ref < 1 || r.min_ref > r.max_ref)) return false;
    return true;
}

int64_t raw_params(const ggns_run_desc &r) {
    const int64_t d = r.d, K = r.n_comp;
    switch (r.lik_kind) {
        case GGNS_LIK_GAUSS_DIAG: return 2 * d;
        case GGNS_LIK_GAUSS_FULL: return d + d * d + 1;
        case GGNS_LIK_SHELLS: return K * (d + 2);
        case GGNS_LIK_TORUS: return 3;
        default: return K * 2 * d;
    }
}

// Coordinates per lane: four (one Philox / xoshiro block of normals per lane)
// unless d is tiny, eight when four would need more than a wavefront.
int default_c(int d) {
    if (d <= 2) return d;
    if (d <= 4 * 64) return 4;
    return 8;
}

struct Plan {
    std::vector<RunDev> runs;
    int64_t off_runs = 0, off_class_runs = 0, off_tiles = 0, n_tile_slots = 0, off_mirror = 0, total = 0;
};

// Lay out the arena: run table, tiles, then each run's arrays.
int make_plan(const ggns_run_desc *descs, int n_runs, Plan &P) {
    if (n_runs < 1 || descs == nullptr) return GGNS_EINVAL;
    P.runs.resize(n_runs);
    int64_t off = 0;
    P.off_runs = off;
    off = align_up(off + (int64_t)sizeof(RunDev) * n_runs);
    // the same descriptors grouped by walk class (each class's runs contiguous),
    // for the per-class iteration chains of ggns_iterate
    P.off_class_runs = off;
    off = align_up(off + (int64_t)sizeof(RunDev) * n_runs);
    // tiles: walk and init tiles of every run (upper bound: one per walker / point)
    int64_t ntiles = 0;
    for (int r = 0; r < n_runs; ++r) ntiles += 2 * (int64_t)descs[r].n_live + 2;
    P.off_tiles = off;
    P.n_tile_slots = ntiles;
    off = align_up(off + (int64_t)sizeof(Tile) * ntiles);
    // contiguous copy of every run's accumulators, gathered for one read-back
    // the stats records the gather packs for one copy to the host
    static_assert(sizeof(ggns_run_stats) <= sizeof(Acc), "stats mirror sized by Acc");
    P.off_mirror = off;
    off = align_up(off + (int64_t)sizeof(Acc) * n_runs);
    for (int r = 0; r < n_runs; ++r) {
        const ggns_run_desc &D = descs[r];
        if (!valid_desc(D)) return GGNS_EINVAL;
        if (D.precision == GGNS_FP32_BF16MMA && D.lik_kind != GGNS_LIK_GAUSS_FULL) return GGNS_EINVAL;
        RunDev &R = P.runs[r];
        std::memset(&R, 0, sizeof(R));
        R.d = D.d; R.n_live = D.n_live; R.n_kill = D.n_kill; R.kind = D.lik_kind;
        R.prec = D.precision; R.n_comp = (D.lik_kind == GGNS_LIK_SHELLS || D.lik_kind == GGNS_LIK_GMM_DIAG) ? D.n_comp : 1;
        R.n_steps_max = D.n_steps_max; R.min_ref = D.min_ref; R.max_ref = D.max_ref;
        R.prune_streak = D.prune_streak; R.term_kind = D.term_kind; R.max_iter = D.max_iter;
        R.lo = D.prior_lo; R.hi = D.prior_hi; R.dt_init = D.dt_init; R.delta_p = D.delta_p;
        R.out_hi = D.out_hi; R.out_lo = D.out_lo; R.dt_down = D.dt_down; R.dt_up = D.dt_up;
        R.term_tol = D.term_tol; R.seed = D.seed; R.param_offset = D.param_offset;
        R.noise_mode = D.noise_mode;
        R.walk_mode = D.walk_mode;
        R.cluster_mode = D.cluster_mode;
        R.cluster_kmax = D.cluster_mode ? D.cluster_kmax : 0;
        const bool mma = D.precision == GGNS_FP32_BF16MMA;
        if (!mma && D.tile_c != 0 && D.tile_c != 1 && D.tile_c != 2 && D.tile_c != 4 && D.tile_c != 8)
            return GGNS_EUNSUPPORTED;
        int C = (D.tile_c && !mma) ? D.tile_c : default_c(D.d);
        int G = next_pow2((D.d + C - 1) / C);
        while (G > 64) { C *= 2; G = next_pow2((D.d + C - 1) / C); }
        if (C > 8 || (D.precision == GGNS_FP64 && C > 4)) return GGNS_EUNSUPPORTED;
        R.C = C; R.G = G;
        R.dp = G * C;
        R.var = lik_variant(D.lik_kind, R.n_comp, D.precision);
        const int64_t es = (D.precision == GGNS_FP64) ? 8 : 4;
        R.nprm = (int32_t)converted_size(R.var, D.d, R.dp);
        const int64_t prm_bytes = (int64_t)R.nprm * es;
        R.nprm_bytes_lds = (prm_bytes <= 48 * 1024) ? (int32_t)prm_bytes : 0;
        // the mixture walk reads its staged block every step (at most
        // kMaxComp (2 kMaxD + 4) doubles = 32.9 KB, so always staged)
        if (R.var == VAR_GMM && R.nprm_bytes_lds == 0) return GGNS_EUNSUPPORTED;
        R.dead_cap = (int64_t)D.n_kill * D.max_iter + D.n_live;
        R.off_acc = off; off = align_up(off + (int64_t)sizeof(Acc));
        R.off_prm = off; off = align_up(off + prm_bytes);
        if (D.precision == GGNS_FP32_BF16MMA) {
            const int64_t dp = (D.d + 31) / 32 * 32;
            // wavefronts per group of 16 walkers: by default eight dimensions per lane
            R.mw = D.tile_c ? D.tile_c : (int32_t)(dp / 32);
            if (!mfma_shape_ok((int)dp, R.mw)) return GGNS_EUNSUPPORTED;
            R.off_prm_bf16 = off; off = align_up(off + dp * dp * 2);
        } else {
            R.off_prm_bf16 = -1;
        }
        R.off_live_x = off; off = align_up(off + (int64_t)D.n_live * D.d * es);
        R.off_live_logl = off; off = align_up(off + (int64_t)D.n_live * 8);
        R.off_killed = off; off = align_up(off + (int64_t)D.n_kill * 4);
        R.off_surv = off; off = align_up(off + (int64_t)(D.n_live - D.n_kill) * 4);
        R.off_surv_sorted = off; off = align_up(off + (int64_t)(D.n_live - D.n_kill) * 4);
        R.off_start = off; off = align_up(off + (int64_t)D.n_kill * 4);
        R.off_walk_x = off; off = align_up(off + (int64_t)D.n_kill * D.d * es);
        R.off_walk_logl = off; off = align_up(off + (int64_t)D.n_kill * 8);
        R.off_dead_logl = off; off = align_up(off + R.dead_cap * 8);
        R.off_dead_logw = off; off = align_up(off + R.dead_cap * 8);
        R.fin_chunks = (int32_t)((R.dead_cap + kFinChunk - 1) / kFinChunk);
        R.off_fin = off; off = align_up(off + (int64_t)R.fin_chunks * 5 * 8);
        if (D.cluster_mode) {
            R.off_label = off; off = align_up(off + (int64_t)D.n_live * 4);
            R.off_cltab = off; off = align_up(off + (int64_t)sizeof(ClusterTab));
            R.off_members = off; off = align_up(off + (int64_t)D.n_live * 4);
            R.off_knn = off; off = align_up(off + (int64_t)D.n_live * kKnnMax * 4);
            R.off_knn_d = off; off = align_up(off + (int64_t)D.n_live * kKnnMax * 8);
            R.off_start_cl = off; off = align_up(off + (int64_t)D.n_kill * 4);
            R.off_knn_part = off; off = align_up(off + (int64_t)D.n_live * kKnnSplit * kKnnPass * 8);
            R.off_knn_part_s = off; off = align_up(off + (int64_t)D.n_live * kKnnSplit * kKnnPass * 4);
        } else {
            R.off_label = R.off_cltab = R.off_members = R.off_knn = R.off_start_cl = -1;
            R.off_knn_d = -1;
            R.off_knn_part = R.off_knn_part_s = -1;
        }
        if (D.walk_mode == 1) {
            // walker states between the two walk launches, over the padded
            // dimension of the run's walk kernel
            const int wdp = mma ? (D.d + 31) / 32 * 32 : (R.dp + 3) / 4 * 4;
            R.wstate_stride = walker_state_bytes(wdp, (int)es);
            R.off_wstate = off; off = align_up(off + (int64_t)D.n_kill * R.wstate_stride);
        } else {
            R.off_wstate = -1;
            R.wstate_stride = 0;
        }
    }
    P.total = off;
    return GGNS_OK;
}

struct Class {
    int prec, C, kind;   // kind: kernel variant (lik_variant)
    bool mfma;
    int64_t tile_off;   // index of the first tile in the arena tile array
    int n_tiles;
    size_t lds;
    int waves = 0;       // matrix-core classes: wavefronts per group of 16 walkers
    int gf = 0;          // vector FP32 walk: lanes per walker (4, 8, 16 or 32) shared by the class, else 0
    bool any_batch = false;   // some run of the class walks the batch-minimum loop
    int nz = 0;               // matrix-core classes: 1 = one noise normal per walker (noise_mode 1)
    // the class's runs: their descriptors start at class_off in the class-ordered
    // run table; the largest n_kill * d and n_live, and their cluster and precision mix
    std::vector<int> runs;
    int class_off = 0, max_kd = 1, max_live = 0;
    bool any_cluster = false, any_fp64 = false, any_fp32 = false;
};

}  // namespace

struct ggns_ctx {
    Plan plan;
    std::vector<ggns_run_desc> descs;
    void *arena = nullptr;
    int64_t arena_bytes = 0;
    const double *params = nullptr;
    int64_t n_params = 0;
    std::vector<Tile> tiles_host;
    std::vector<Class> walk_classes, init_classes;
    int n_simd = 1024;   // SIMDs of the device (256 compute units x 4 on MI355X)
    int max_kd = 1;
    bool any_cluster = false, any_fp64 = false, any_fp32 = false;
    int max_live = 0;
    // walk classes after the first run on side streams forked from and joined
    // back into the caller's stream (default priority; capturable)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;

    ~ggns_ctx() {
        for (hipStream_t s : side) (void)hipStreamDestroy(s);
        for (hipEvent_t e : join) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
    }

    // the run descriptors grouped by walk class (host copy of the device table)
    // and each run's position in it
    std::vector<RunDev> class_table;
    std::vector<int> class_pos;

    RunDev *runs_dev() const { return at<RunDev>(arena, plan.off_runs); }
    RunDev *class_runs_dev() const { return at<RunDev>(arena, plan.off_class_runs); }
    Tile *tiles_dev() const { return at<Tile>(arena, plan.off_tiles); }
};

namespace {

// Walk tiles: one walker per lane group, kWalkThreads / G groups per block.
// Init tiles: the same shape over the n_live prior draws.
void build_classes(ggns_ctx *c) {
    // (prec, C, kind, fixed group size) -> runs; FP32 runs with groups of 4, 8, 16
    // or 32 lanes get a kernel with that size fixed at compile time
    std::map<std::tuple<int, int, int, int>, std::vector<int>> groups;
    std::vector<int> mfma_runs;
    for (int r = 0; r < (int)c->plan.runs.size(); ++r) {
        const RunDev &R = c->plan.runs[r];
        if (R.prec == GGNS_FP32_BF16MMA)
            mfma_runs.push_back(r);
        else
            groups[std::make_tuple(R.prec, R.C, R.var,
                                   (R.prec == GGNS_FP32 && (R.G == 4 || R.G == 8 || R.G == 16 || R.G == 32)) ? R.G : 0)]
                .push_back(r);
        c->max_kd = std::max<int>(c->max_kd, R.n_kill * R.d);
    }
    c->tiles_host.clear();
    auto add_tiles = [&](int r, int count, int per) {
        for (int b = 0; b < count; b += per) {
            Tile t;
            t.run = r; t.m_begin = b; t.m_end = std::min(count, b + per); t.pad = 0;
            c->tiles_host.push_back(t);
        }
    };
    for (auto &kv : groups) {
        Class w{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), false,
                (int64_t)c->tiles_host.size(), 0, 0};
        w.gf = std::get<3>(kv.first);
        size_t lds = 0;
        for (int r : kv.second) {
            const RunDev &R = c->plan.runs[r];
            add_tiles(r, R.n_kill, kWalkThreads / R.G);
            size_t need = (size_t)((R.nprm_bytes_lds + 15) & ~15);
            if (R.kind == GGNS_LIK_GAUSS_FULL)
                need += (size_t)kWalkThreads * R.C * (R.prec == GGNS_FP64 ? 8 : 4);
            lds = std::max(lds, need);
        }
        w.n_tiles = (int)(c->tiles_host.size() - w.tile_off);
        w.lds = lds;
        w.runs = kv.second;
        for (int r : kv.second) w.any_batch = w.any_batch || c->plan.runs[r].walk_mode == 1;
        // the mixture kernel that holds its means and precisions in registers
        // runs two wavefronts per SIMD; a class with more wavefronts than that
        // fills the device with is bound by occupancy, and its kernel reads
        // the staged block every step instead (three wavefronts per SIMD)
        if (w.kind == VAR_GMM) {
            int64_t waves = 0;
            for (int r : kv.second)
                waves += ((int64_t)c->plan.runs[r].n_kill * c->plan.runs[r].G + 63) / 64;
            if (waves > 2 * (int64_t)c->n_simd) w.kind = VAR_GMM_STAGED;
        }
        c->walk_classes.push_back(w);
    }
    for (auto &kv : groups) {
        Class w{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), false,
                (int64_t)c->tiles_host.size(), 0, 0};
        w.lds = (size_t)kWalkThreads * w.C * (w.prec == GGNS_FP64 ? 8 : 4);
        for (int r : kv.second) add_tiles(r, c->plan.runs[r].n_live, kWalkThreads / c->plan.runs[r].G);
        w.n_tiles = (int)(c->tiles_host.size() - w.tile_off);
        c->init_classes.push_back(w);
    }
    if (!mfma_runs.empty()) {
        // matrix-core walk: one class per (padded dimension, wavefronts per
        // group), 16 walkers per tile (one group of slots)
        std::map<std::tuple<int, int, int>, std::vector<int>> by_dp;
        for (int r : mfma_runs)
            by_dp[std::make_tuple((c->plan.runs[r].d + 31) / 32 * 32, c->plan.runs[r].mw,
                                  c->plan.runs[r].noise_mode != 0 ? 1 : 0)]
                .push_back(r);
        for (auto &kv : by_dp) {
            Class w{GGNS_FP32_BF16MMA, std::get<0>(kv.first), GGNS_LIK_GAUSS_FULL, true,
                    (int64_t)c->tiles_host.size(), 0, 0};
            w.waves = std::get<1>(kv.first);
            w.nz = std::get<2>(kv.first);
            for (int r : kv.second) {
                add_tiles(r, c->plan.runs[r].n_kill, 16);
                w.any_batch = w.any_batch || c->plan.runs[r].walk_mode == 1;
            }
            w.n_tiles = (int)(c->tiles_host.size() - w.tile_off);
            w.runs = kv.second;
            c->walk_classes.push_back(w);
        }
        // prior draws of MMA runs on the FP32 vector path (one class per C)
        for (int r : mfma_runs) {
            Class i{GGNS_FP32, c->plan.runs[r].C, VAR_GAUSS_FULL_BF16, false,
                    (int64_t)c->tiles_host.size(), 0, 0};
            add_tiles(r, c->plan.runs[r].n_live, kWalkThreads / c->plan.runs[r].G);
            i.n_tiles = (int)(c->tiles_host.size() - i.tile_off);
            c->init_classes.push_back(i);
        }
    }
}

int create(ggns_ctx **out, const ggns_run_desc *runs, int32_t n_runs, const double *params_dev,
           int64_t n_params, void *arena, int64_t arena_bytes, void *stream, bool fresh) {
    if (out == nullptr || arena == nullptr || params_dev == nullptr) return GGNS_EINVAL;
    *out = nullptr;
    ggns_ctx *c = new ggns_ctx();
    int rc = make_plan(runs, n_runs, c->plan);
    if (rc != GGNS_OK) { delete c; return rc; }
    if (arena_bytes < c->plan.total || (reinterpret_cast<uintptr_t>(arena) % kAlign) != 0) {
        delete c;
        return GGNS_EINVAL;
    }
    for (int r = 0; r < n_runs; ++r) {
        if (runs[r].param_offset + raw_params(runs[r]) > n_params) { delete c; return GGNS_EINVAL; }
    }
    // the fixed scratch buffer's address on this device, taken here once per
    // device so that ggns_hss_walk_plain_static only reads a table
    if (scratch_for_current_device() == nullptr) { delete c; return GGNS_EHIP; }
    c->descs.assign(runs, runs + n_runs);
    c->arena = arena;
    c->arena_bytes = arena_bytes;
    c->params = params_dev;
    c->n_params = n_params;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0)
            c->n_simd = 4 * cus;   // four SIMDs per compute unit
    }
    build_classes(c);
    // every run belongs to exactly one walk class: lay the descriptors out class
    // by class and note what each class's chain of launches needs
    std::vector<RunDev> &class_table = c->class_table;
    c->class_pos.assign(n_runs, -1);
    for (Class &w : c->walk_classes) {
        w.class_off = (int)class_table.size();
        for (int r : w.runs) {
            const RunDev &R = c->plan.runs[r];
            c->class_pos[r] = (int)class_table.size();
            class_table.push_back(R);
            w.max_kd = std::max<int>(w.max_kd, R.n_kill * R.d);
            if (R.cluster_mode) {
                w.any_cluster = true;
                w.max_live = std::max(w.max_live, R.n_live);
                if (R.prec == GGNS_FP64) w.any_fp64 = true; else w.any_fp32 = true;
            }
        }
    }
    if ((int)class_table.size() != n_runs) { delete c; return GGNS_EINVAL; }
    for (const RunDev &R : c->plan.runs) {
        if (R.cluster_mode) {
            c->any_cluster = true;
            c->max_live = std::max(c->max_live, R.n_live);
            if (R.prec == GGNS_FP64) c->any_fp64 = true; else c->any_fp32 = true;
        }
    }
    for (size_t i = 1; i < c->walk_classes.size(); ++i) {
        hipStream_t ss;
        hipEvent_t e;
        if (hipStreamCreateWithFlags(&ss, hipStreamNonBlocking) != hipSuccess) { delete c; return GGNS_EHIP; }
        c->side.push_back(ss);
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { delete c; return GGNS_EHIP; }
        c->join.push_back(e);
    }
    if (c->walk_classes.size() > 1 &&
        hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return GGNS_EHIP;
    }
    // MMA runs convert P to FP32 too: their prior draws and the stand-alone
    // likelihood use the FP32 vector path
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(c->runs_dev(), c->plan.runs.data(), sizeof(RunDev) * n_runs,
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c->class_runs_dev(), class_table.data(), sizeof(RunDev) * n_runs,
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c->tiles_dev(), c->tiles_host.data(), sizeof(Tile) * c->tiles_host.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess) {
        delete c;
        return GGNS_EHIP;
    }
    launch_prepare(arena, c->runs_dev(), n_runs, params_dev, s, fresh ? 1 : 0);
    if (hipGetLastError() != hipSuccess) { delete c; return GGNS_EHIP; }
    if (fresh) {
        for (const Class &w : c->init_classes) {
            rc = launch_init_class(arena, c->runs_dev(), c->tiles_dev() + w.tile_off, w.n_tiles,
                                   w.prec == GGNS_FP64 ? GGNS_FP64 : GGNS_FP32, w.C, w.kind, s);
            if (rc != GGNS_OK) { delete c; return rc; }
        }
    }
    *out = c;
    return GGNS_OK;
}

}  // namespace

namespace ggns {
int64_t walker_state_bytes(int d_pad, int elem_bytes) {
    // x, p and the fallback point (elem_bytes each), one noise stream word per
    // coordinate (four per block of four), the reservoir stream (16 bytes),
    // six counters and the fallback log L, padded to 80 bytes
    return (int64_t)(3 * elem_bytes + 4) * d_pad + 80;
}
}  // namespace ggns

namespace {
// One class's walk: a class with batch-minimum runs walks twice, the first walk
// fixing each run's window and the second finishing every run of the class.
int walk_class(const ggns_ctx *ctx, const Class &w, hipStream_t st) {
    auto phase = [&](int ph) {
        if (w.mfma)
            return launch_walk_mfma(ctx->arena, ctx->runs_dev(), ctx->tiles_dev() + w.tile_off,
                                    w.n_tiles, w.C, w.waves, w.nz, ph, st);
        return launch_walk_class(ctx->arena, ctx->runs_dev(), ctx->tiles_dev() + w.tile_off,
                                 w.n_tiles, w.prec, w.C, w.kind, w.gf, w.lds, ph, st);
    };
    if (w.any_batch) {
        const int rc = phase(1);
        if (rc != GGNS_OK) return rc;
    }
    return phase(2);
}

// Runs `body(class, stream)` for every walk class: the first on the caller's
// stream, the others on side streams forked from it and joined back into it.
// Classes own disjoint runs, so their work is independent.
template <typename F>
int fork_classes(ggns_ctx *ctx, hipStream_t s, F body) {
    const size_t n = ctx->walk_classes.size();
    if (n == 0) return GGNS_OK;
    if (n == 1) return body(ctx->walk_classes[0], s);
    if (hipEventRecord(ctx->fork, s) != hipSuccess) return GGNS_EHIP;
    for (size_t i = 1; i < n; ++i) {
        if (hipStreamWaitEvent(ctx->side[i - 1], ctx->fork, 0) != hipSuccess) return GGNS_EHIP;
        const int rc = body(ctx->walk_classes[i], ctx->side[i - 1]);
        if (rc != GGNS_OK) return rc;
        if (hipEventRecord(ctx->join[i - 1], ctx->side[i - 1]) != hipSuccess) return GGNS_EHIP;
    }
    const int rc = body(ctx->walk_classes[0], s);
    for (size_t i = 1; i < n; ++i)
        if (hipStreamWaitEvent(s, ctx->join[i - 1], 0) != hipSuccess) return GGNS_EHIP;
    return rc;
}
}  // namespace

extern "C" {

int64_t ggns_arena_bytes(const ggns_run_desc *runs, int32_t n_runs) {
    Plan P;
    const int rc = make_plan(runs, n_runs, P);
    return rc == GGNS_OK ? P.total : (int64_t)rc;
}

int ggns_init(ggns_ctx **out, const ggns_run_desc *runs, int32_t n_runs, const double *params_dev,
              int64_t n_params, void *arena_dev, int64_t arena_bytes, void *stream) {
    return create(out, runs, n_runs, params_dev, n_params, arena_dev, arena_bytes, stream, true);
}

int ggns_attach(ggns_ctx **out, const ggns_run_desc *runs, int32_t n_runs, const double *params_dev,
                int64_t n_params, void *arena_dev, int64_t arena_bytes, void *stream) {
    return create(out, runs, n_runs, params_dev, n_params, arena_dev, arena_bytes, stream, false);
}

int ggns_evidence_update(ggns_ctx *ctx, int32_t final_sweep, void *stream) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (ctx->any_cluster) {
        const int rc = launch_clusters(ctx->arena, ctx->runs_dev(), (int)ctx->plan.runs.size(),
                                       ctx->max_live, final_sweep ? 1 : 0, ctx->any_fp64,
                                       ctx->any_fp32, reinterpret_cast<hipStream_t>(stream));
        if (rc != GGNS_OK) return rc;
    }
    launch_evidence(ctx->arena, ctx->runs_dev(), (int)ctx->plan.runs.size(), final_sweep ? 1 : 0,
                    ctx->any_cluster ? 1 : 0, reinterpret_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

int ggns_finalize(ggns_ctx *ctx, void *stream) {
    if (ctx == nullptr) return GGNS_ESTATE;
    int max_chunks = 1;
    for (const RunDev &R : ctx->plan.runs) max_chunks = std::max(max_chunks, (int)R.fin_chunks);
    launch_finalize(ctx->arena, ctx->runs_dev(), (int)ctx->plan.runs.size(), max_chunks,
                    reinterpret_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

int ggns_hss_walk(ggns_ctx *ctx, void *stream) {
    if (ctx == nullptr) return GGNS_ESTATE;
    return fork_classes(ctx, reinterpret_cast<hipStream_t>(stream),
                        [&](const Class &w, hipStream_t st) { return walk_class(ctx, w, st); });
}

int ggns_iterate(ggns_ctx *ctx, int32_t n_iter, void *stream) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (n_iter < 0) return GGNS_EINVAL;
    if (n_iter == 0) return GGNS_OK;
    // each class runs its own chain of iterations over its own runs; the work of
    // one run is that of the one-call-per-iteration sequence, launch for launch
    return fork_classes(ctx, reinterpret_cast<hipStream_t>(stream), [&](const Class &w, hipStream_t st) -> int {
        RunDev *cr = ctx->class_runs_dev() + w.class_off;
        const int nr = (int)w.runs.size();
        for (int it = 0; it < n_iter; ++it) {
            if (w.any_cluster) {
                const int rc = launch_clusters(ctx->arena, cr, nr, w.max_live, 0, w.any_fp64,
                                               w.any_fp32, st);
                if (rc != GGNS_OK) return rc;
            }
            launch_evidence(ctx->arena, cr, nr, 0, w.any_cluster ? 1 : 0, st);
            const int rc = walk_class(ctx, w, st);
            if (rc != GGNS_OK) return rc;
            launch_replace(ctx->arena, cr, nr, w.max_kd, st);
        }
        return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
    });
}

int64_t ggns_plain_workspace_bytes(const ggns_ctx *ctx) {
    if (ctx == nullptr) return GGNS_ESTATE;
    int64_t b = 0;
    for (const RunDev &R : ctx->plan.runs) b = std::max(b, plain_workspace_bytes(R));
    return b;
}

int ggns_hss_walk_plain(ggns_ctx *ctx, void *workspace_dev, int64_t workspace_bytes, void *stream) {
    if (ctx == nullptr) return GGNS_ESTATE;
    for (const RunDev &R : ctx->plan.runs)
        if (R.prec != GGNS_FP64) return GGNS_EUNSUPPORTED;
    if (workspace_dev == nullptr || (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign) != 0 ||
        workspace_bytes < ggns_plain_workspace_bytes(ctx))
        return GGNS_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (int r = 0; r < (int)ctx->plan.runs.size(); ++r) {
        const int rc = launch_walk_plain(ctx->arena, ctx->runs_dev(), r, ctx->plan.runs[r],
                                         workspace_dev, 8, s);
        if (rc != GGNS_OK) return rc;
    }
    return GGNS_OK;
}

int ggns_hss_walk_plain_static(ggns_ctx *ctx, void *stream) {
    if (ctx == nullptr) return GGNS_ESTATE;
    for (const RunDev &R : ctx->plan.runs)
        if (R.prec != GGNS_FP64) return GGNS_EUNSUPPORTED;
    if (ggns_plain_workspace_bytes(ctx) > GGNS_STATIC_SCRATCH_BYTES) return GGNS_ESCRATCH;
    void *ws = scratch_for_current_device();
    if (ws == nullptr) return GGNS_EHIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (int r = 0; r < (int)ctx->plan.runs.size(); ++r) {
        const int rc = launch_walk_plain(ctx->arena, ctx->runs_dev(), r, ctx->plan.runs[r], ws, 8, s);
        if (rc != GGNS_OK) return rc;
    }
    return GGNS_OK;
}

namespace {
int ext_check(const ggns_ctx *ctx, int32_t run, const void *ws, int64_t bytes) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (run < 0 || run >= (int)ctx->plan.runs.size()) return GGNS_EINVAL;
    if (ctx->plan.runs[run].prec != GGNS_FP64) return GGNS_EUNSUPPORTED;
    if (ws == nullptr || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 ||
        bytes < plain_workspace_bytes(ctx->plan.runs[run]))
        return GGNS_EINVAL;
    return GGNS_OK;
}
}  // namespace

int64_t ggns_ext_workspace_bytes(const ggns_ctx *ctx, int32_t run) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (run < 0 || run >= (int)ctx->plan.runs.size()) return GGNS_EINVAL;
    return plain_workspace_bytes(ctx->plan.runs[run]);
}

int ggns_ext_buffers(const ggns_ctx *ctx, int32_t run, void *workspace_dev, int64_t workspace_bytes,
                     double **x_dev, double **logl_dev, double **grad_dev, int32_t **active_dev) {
    const int rc = ext_check(ctx, run, workspace_dev, workspace_bytes);
    if (rc != GGNS_OK) return rc;
    if (!x_dev || !logl_dev || !grad_dev || !active_dev) return GGNS_EINVAL;
    ext_buffers(ctx->plan.runs[run], workspace_dev, x_dev, logl_dev, grad_dev, active_dev);
    return GGNS_OK;
}

int ggns_ext_begin(ggns_ctx *ctx, int32_t run, void *workspace_dev, int64_t workspace_bytes,
                   void *stream) {
    const int rc = ext_check(ctx, run, workspace_dev, workspace_bytes);
    if (rc != GGNS_OK) return rc;
    return launch_ext_begin(ctx->arena, ctx->runs_dev(), run, ctx->plan.runs[run], workspace_dev,
                            reinterpret_cast<hipStream_t>(stream));
}

int ggns_ext_step(ggns_ctx *ctx, int32_t run, void *workspace_dev, int64_t workspace_bytes,
                  int32_t step, void *stream) {
    const int rc = ext_check(ctx, run, workspace_dev, workspace_bytes);
    if (rc != GGNS_OK) return rc;
    // the batch-minimum loop takes one call more (step == n_steps_max): the
    // save rule of the last step
    const RunDev &R = ctx->plan.runs[run];
    if (step < 0 || step >= R.n_steps_max + (R.walk_mode == 1 ? 1 : 0)) return GGNS_EINVAL;
    return launch_ext_step(ctx->arena, ctx->runs_dev(), run, ctx->plan.runs[run], workspace_dev, step,
                           reinterpret_cast<hipStream_t>(stream));
}

int ggns_replace_dead(ggns_ctx *ctx, void *stream) {
    if (ctx == nullptr) return GGNS_ESTATE;
    launch_replace(ctx->arena, ctx->runs_dev(), (int)ctx->plan.runs.size(), ctx->max_kd,
                   reinterpret_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

int ggns_loglike_grad(ggns_ctx *ctx, int32_t run, const void *x_dev, int64_t n, double *logl_dev,
                      void *grad_dev, void *stream) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (run < 0 || run >= (int)ctx->plan.runs.size() || n < 0 || (n > 0 && x_dev == nullptr))
        return GGNS_EINVAL;
    if (n == 0) return GGNS_OK;
    return launch_loglike(ctx->arena, ctx->runs_dev() + run, ctx->plan.runs[run], x_dev, n,
                          logl_dev, grad_dev, nullptr, reinterpret_cast<hipStream_t>(stream));
}

int ggns_loglike_vjp(ggns_ctx *ctx, int32_t run, const void *x_dev, int64_t n,
                     const double *gout_dev, void *gx_dev, void *stream) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (run < 0 || run >= (int)ctx->plan.runs.size() || n < 0 ||
        (n > 0 && (x_dev == nullptr || gout_dev == nullptr || gx_dev == nullptr)))
        return GGNS_EINVAL;
    if (n == 0) return GGNS_OK;
    return launch_loglike(ctx->arena, ctx->runs_dev() + run, ctx->plan.runs[run], x_dev, n,
                          nullptr, gx_dev, gout_dev, reinterpret_cast<hipStream_t>(stream));
}

int ggns_run_layout(const ggns_ctx *ctx, int32_t run, ggns_layout *out) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (run < 0 || run >= (int)ctx->plan.runs.size() || out == nullptr) return GGNS_EINVAL;
    const RunDev &R = ctx->plan.runs[run];
    out->live_x = R.off_live_x;
    out->live_logl = R.off_live_logl;
    out->killed = R.off_killed;
    out->survivors = R.off_surv;
    out->start = R.off_start;
    out->walk_x = R.off_walk_x;
    out->walk_logl = R.off_walk_logl;
    out->dead_logl = R.off_dead_logl;
    out->dead_logw = R.off_dead_logw;
    out->dead_cap = R.dead_cap;
    out->elem_bytes = (R.prec == GGNS_FP64) ? 8 : 4;
    out->reserved = 0;
    out->label = R.off_label;
    out->cluster_table = R.off_cltab;
    out->knn = R.off_knn;
    out->knn_dist = R.off_knn_d;
    return GGNS_OK;
}

int ggns_read_stats_async(ggns_ctx *ctx, ggns_run_stats *out, void *stream) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (out == nullptr) return GGNS_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int n = (int)ctx->plan.runs.size();
    ggns_run_stats *mirror = at<ggns_run_stats>(ctx->arena, ctx->plan.off_mirror);
    if (launch_gather_acc(ctx->arena, ctx->runs_dev(), n, mirror, s) != GGNS_OK ||
        hipMemcpyAsync(out, mirror, sizeof(ggns_run_stats) * n, hipMemcpyDeviceToHost, s) !=
            hipSuccess)
        return GGNS_EHIP;
    return GGNS_OK;
}

int ggns_read_stats(ggns_ctx *ctx, ggns_run_stats *out, void *stream) {
    const int rc = ggns_read_stats_async(ctx, out, stream);
    if (rc != GGNS_OK) return rc;
    return hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? GGNS_OK
                                                                                     : GGNS_EHIP;
}

int ggns_write_vars(ggns_ctx *ctx, int32_t run, const ggns_run_vars *v, void *stream) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (run < 0 || run >= (int)ctx->plan.runs.size() || v == nullptr) return GGNS_EINVAL;
    launch_set_vars(ctx->arena, ctx->runs_dev() + run, v->log_z, v->log_x, v->dt, (long long)v->iter,
                    reinterpret_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

namespace {
// Both device copies of one run's descriptor after a host-side change.
int upload_run(ggns_ctx *ctx, int run) {
    const RunDev &R = ctx->plan.runs[run];
    ctx->class_table[ctx->class_pos[run]] = R;
    if (hipMemcpy(ctx->runs_dev() + run, &R, sizeof(RunDev), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->class_runs_dev() + ctx->class_pos[run], &R, sizeof(RunDev),
                  hipMemcpyHostToDevice) != hipSuccess)
        return GGNS_EHIP;
    return GGNS_OK;
}
}  // namespace

int ggns_set_trace(ggns_ctx *ctx, int32_t run, void *trace_x, double *trace_logl,
                   int32_t *trace_out, int32_t trace_steps) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (run < 0 || run >= (int)ctx->plan.runs.size() || trace_steps < 0) return GGNS_EINVAL;
    if (trace_x != nullptr && (trace_logl == nullptr || trace_out == nullptr)) return GGNS_EINVAL;
    RunDev &R = ctx->plan.runs[run];
    R.trace_x = trace_x;
    R.trace_logl = trace_x ? trace_logl : nullptr;
    R.trace_out = trace_x ? trace_out : nullptr;
    R.trace_steps = trace_x ? trace_steps : 0;
    return upload_run(ctx, run);
}

int ggns_set_dead_x(ggns_ctx *ctx, int32_t run, void *dead_x_dev, int64_t capacity_rows) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (run < 0 || run >= (int)ctx->plan.runs.size() || capacity_rows < 0) return GGNS_EINVAL;
    RunDev &R = ctx->plan.runs[run];
    R.dead_x = (capacity_rows > 0) ? dead_x_dev : nullptr;
    R.dead_x_cap = (dead_x_dev != nullptr) ? capacity_rows : 0;
    return upload_run(ctx, run);
}

int ggns_tile_shape(const ggns_ctx *ctx, int32_t run, int32_t *coords_per_lane,
                    int32_t *lanes_per_walker) {
    if (ctx == nullptr) return GGNS_ESTATE;
    if (run < 0 || run >= (int)ctx->plan.runs.size()) return GGNS_EINVAL;
    const RunDev &R = ctx->plan.runs[run];
    if (R.prec == GGNS_FP32_BF16MMA) {
        const int dp = (R.d + 31) / 32 * 32;
        if (coords_per_lane) *coords_per_lane = dp / (4 * R.mw);
        if (lanes_per_walker) *lanes_per_walker = 4 * R.mw;
    } else {
        if (coords_per_lane) *coords_per_lane = R.C;
        if (lanes_per_walker) *lanes_per_walker = R.G;
    }
    return GGNS_OK;
}

int ggns_noise_normals(uint64_t seed, int32_t iteration, int32_t n_walkers, int32_t n_blocks,
                       int32_t steps, float *normals_dev, uint32_t *words_dev, float *checksum_dev,
                       void *stream) {
    if (n_walkers < 0 || n_blocks < 0 || steps < 0 || iteration < 0) return GGNS_EINVAL;
    const int64_t total = (int64_t)n_walkers * n_blocks;
    if (total > (int64_t)1 << 30 || total * steps * 4 > ((int64_t)1 << 40)) return GGNS_EINVAL;
    return launch_noise_normals(seed, iteration, n_walkers, n_blocks, steps, normals_dev, words_dev,
                                checksum_dev, reinterpret_cast<hipStream_t>(stream));
}

void ggns_free(ggns_ctx *ctx) { delete ctx; }

const char *ggns_status_string(int code) {
    switch (code) {
        case GGNS_OK: return "ok";
        case GGNS_EINVAL: return "invalid argument";
        case GGNS_EHIP: return "HIP error";
        case GGNS_EUNSUPPORTED: return "unsupported size or combination";
        case GGNS_ESTATE: return "invalid state";
        case GGNS_ESCRATCH: return "run too large for the library's fixed scratch buffer";
    }
    return "unknown status";
}

}  // extern "C"
