// capi.hip -- the C ABI: contexts, schedule tables, argument checks, solves.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "dataflow.hpp"

namespace ccp {

// ----- error reporting -----------------------------------------------------
static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

// ----- kernels (sweep.hip, resid.hip) --------------------------------------
template <typename T> int launch_sweep_round(const Tile *, int, int, int64_t, T *, const T *, T *, hipStream_t);
template <typename T> int set_sweep_lds_limits(int);
template <typename T, typename DT> int launch_pair_pass(int64_t, T *, T *, T *, const T *, const DT *, hipStream_t);
template <typename T> int launch_prepare(int64_t, const double *, double, T *, int *, hipStream_t);
template <typename T> int launch_init_cold(int64_t, int64_t, T *, T *, T *, T *, double, hipStream_t);
template <typename S, typename D> int launch_convert(int64_t, const S *, D *, hipStream_t);
template <typename T> int launch_nearness_init(int64_t, int64_t, const double *, T *, T *, hipStream_t);
template <typename T>
int launch_nearness_pair_resid(int64_t, const T *, const double *, const double *, const double *, double *,
                               hipStream_t);
template <typename T> int launch_metric_resid(const Tile *, const int32_t *, int64_t, int, int64_t, const T *, const T *, double *, hipStream_t);
template <typename T, typename DT> int launch_pair_resid(int64_t, const T *, const T *, const T *, const double *, const DT *, const double *, double, double *, hipStream_t);
int launch_final_reduce(const double *, int64_t, const double *, double *, hipStream_t);
int pair_partial_blocks();
int launch_weight_classes(int64_t, const double *, const uint8_t *, double *, hipStream_t);
template <typename T> int launch_aty_round(const Tile *, int, int, int64_t, const T *, double *, hipStream_t);
template <typename T> int launch_x_from_aty(int64_t, const double *, const T *, const double *, double, T *, T *, hipStream_t);
template <typename T> int launch_to_lex(const Tile *, int64_t, int, int64_t, const T *, T *, hipStream_t);
int launch_slots_to_lex(const Tile *, int64_t, int, int64_t, const int64_t *, int64_t, int64_t *, hipStream_t);


void build_dataflow_tables(int64_t n, int b, std::vector<DTile> &tiles, std::vector<uint32_t> &needs,
                           std::vector<uint32_t> &K);
template <typename T> int launch_sweep_dataflow(const DataflowArgs &, int, int, int64_t, T *, const T *, T *, void *, const CompactArgs<T> *, hipStream_t);
template <typename T> int launch_compact_to_slots(int, int64_t, const uint16_t *, const T *, const int64_t *, const uint32_t *, T *, hipStream_t);
template <typename T> int launch_compact_export(int, int64_t, int, const DTile *, const int32_t *, const uint16_t *, const T *, const int64_t *, const uint32_t *, int64_t *, T *, hipStream_t);
template <typename T> int launch_mask_build(int, int64_t, const T *, void *, hipStream_t);
template <typename T> int launch_sweep_colour(int64_t, T *, const T *, T *, hipStream_t);
template <typename T> int dataflow_occupancy(int, int *);
template <typename T> int launch_aty_dataflow(const DataflowArgs &, int, int, int64_t, const T *, double *, hipStream_t);
int launch_dataflow_reset(uint32_t *, hipStream_t);
template <typename T>
int launch_infer_aty_dataflow(const DataflowArgs &, int, const GraphView &, const float *, T *, double *, hipStream_t);
template <typename T> int infer_aty_occupancy(int, int *);
template <typename T> int aty_dataflow_occupancy(int, int *);
int launch_fill_u32(int64_t, uint32_t *, hipStream_t);

int mlp_num_params();
size_t mlp_workspace_bytes(int64_t count);
int mlp_grad_blocks(int64_t count);
int launch_mlp_train_explicit(const float *, const float *, int64_t, float *, float *, float *, int,
                              float, float *, void *, float *, hipStream_t);
template <typename T>
int launch_mlp_train_graph(const GraphView &, const T *, int64_t, uint64_t, int64_t, float *, float *,
                           float *, int, float, void *, float *, hipStream_t);
int launch_mlp_forward(const float *, const float *, int64_t, float *, hipStream_t);
template <typename T> int launch_mlp_infer(const GraphView &, const float *, T *, hipStream_t);
int launch_mlp_slot_features(const GraphView &, const int64_t *, int64_t, float *, hipStream_t);
int launch_mean_deg(const float *, int64_t, float *, hipStream_t);
template <typename T>
int launch_gate_sample_aty(const GraphView &, const float *, const int64_t *, int64_t, double *, hipStream_t);
template <typename T>
int launch_gate_pairs(int64_t, int64_t, const int64_t *, const double *, const uint8_t *, const T *, double *, uint8_t *, T *,
                      hipStream_t);
template <typename T>
int launch_gate_delta(int64_t, const double *, const T *, const T *, const double *, const uint8_t *, double, double *,
                      hipStream_t);

}  // namespace ccp

using namespace ccp;

struct cc_ctx {
    int64_t n = 0;
    int b = 0;
    int prec = CC_F64;
    hipStream_t stream = nullptr;
    int nb = 0;
    int nrounds = 0;
    int64_t ntiles = 0;
    int64_t slots = 0;
    std::vector<int64_t> round_start;  // tiles of round r: [round_start[r], round_start[r+1])
    Tile *d_tiles = nullptr;
    double *d_mpart = nullptr;  // metric residual partials, 4 per chunk
    double *d_ppart = nullptr;  // pair residual partials
    double *d_out = nullptr;    // final reduction, 14 doubles
    int *d_flag = nullptr;
    double *d_ax = nullptr;     // A'y accumulator, N_p doubles (allocated on first use)
    // dataflow executor (built on first use)
    DTile *d_dtiles = nullptr;
    uint32_t *d_needs = nullptr;
    uint32_t *d_K = nullptr;
    uint32_t *d_cnt = nullptr;   // completed touches per block
    uint32_t *d_ctl = nullptr;   // ticket counter, abort flag
    int64_t nblocks = 0;
    uint32_t kmax = 0;
    uint32_t epoch = 0;
    // workgroups of the dataflow sweeps: a fixed count (0: the defaults),
    // the defaults of the dense and of the sparse / compacted sweeps, and
    // the most that are resident at once (occupancy x CUs, one per tile)
    int df_grid_fixed = 0;
    int df_grid_dense = 0;
    int df_grid_sparse = 0;
    int df_grid_cap = 0;
    int aty_grid = 0;
    int iad_grid = 0;  // workgroups of the fused inference + A'y launch
    uint64_t wait_ticks = 0;
    float *d_mean_deg = nullptr;  // warm-start features
    int32_t *d_chunks = nullptr;  // (tile, first step) per chunk of kChunkSteps tile steps
    int64_t nchunks = 0;
    // compacted dual lists (allocated by cc_compact_init)
    uint16_t *cp_idx[2] = {nullptr, nullptr};
    void *cp_val[2] = {nullptr, nullptr};
    int64_t cp_cap[2] = {0, 0};
    int64_t *cp_off[2] = {nullptr, nullptr};
    uint32_t *cp_cnt[2] = {nullptr, nullptr};
    int cp_cur = 0;                      // the pool holding the current lists
    unsigned long long *cp_alloc = nullptr;
    uint32_t *cp_flag = nullptr;
    void *cp_xsnap = nullptr;            // x before the sweep, for a repeat
    int32_t *cp_step_tile = nullptr;     // tile of each tile step (export)
    int64_t cp_nnz = 0;                  // entries after the last sweep
    int cp_regrows = 0;                  // sweeps repeated with a larger pool
    // sampled warm-start gate: pairs to draw (0: off), and what the last
    // warm start drew, estimated and decided
    int64_t gate_sample = 16384;
    int64_t gate_drawn = 0;
    double gate_gain = 0.0, gate_se = 0.0;
    int gate_rejected = 0;
};

namespace {

int64_t num_pairs(int64_t n) { return n * (n - 1) / 2; }
size_t elem_size(const cc_ctx *c) { return c->prec == CC_F64 ? sizeof(double) : sizeof(float); }

int check_ctx(const cc_ctx *c) {
    if (!c) return fail(CC_EINVAL, "null context");
    return CC_OK;
}

int need(const void *p, const char *name) {
    if (!p) return fail(CC_EINVAL, std::string("null pointer: ") + name);
    return CC_OK;
}

// Scratch allocation released at scope exit.
struct DevTmp {
    void *p = nullptr;
    ~DevTmp() { if (p) (void)hipFree(p); }
    int alloc(size_t bytes) {
        if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) {
            p = nullptr;
            return fail(CC_ENOMEM, "hipMalloc of scratch failed");
        }
        return CC_OK;
    }
};

// Build the tiled schedule (Sec. III-C): tiles in round order, rounds the
// block anti-diagonals s = nb-1 .. 0 followed by s = nb .. 2nb-2, tiles of
// a round by ascending P.  Each tile's dual segment holds
// (Q-P+1) * b sub-steps * 3 orientations * b*b lanes.
void build_schedule(cc_ctx *c, std::vector<Tile> &tiles) {
    const int nb = c->nb;
    const int64_t bb = int64_t(c->b) * c->b;
    int64_t ybase = 0;
    c->round_start.clear();
    for (int r = 0; r < c->nrounds; ++r) {
        c->round_start.push_back(int64_t(tiles.size()));
        const int s = (r < nb) ? (nb - 1 - r) : r;
        for (int P = 0; 2 * P <= s; ++P) {
            const int Q = s - P;
            if (Q >= nb) continue;
            tiles.push_back(Tile{P, Q, ybase});
            ybase += int64_t(Q - P + 1) * c->b * 3 * bb;
        }
    }
    c->round_start.push_back(int64_t(tiles.size()));
    c->ntiles = int64_t(tiles.size());
    c->slots = ybase;
}

template <typename T>
int sweep_rounds_t(cc_ctx *c, T *x, T *y, const T *g, int first, int count) {
    for (int r = first; r < first + count; ++r) {
        const int64_t a = c->round_start[r], e = c->round_start[r + 1];
        int rc = launch_sweep_round<T>(c->d_tiles + a, int(e - a), c->b, c->n, x, g, y, c->stream);
        if (rc) return rc;
    }
    return CC_OK;
}

template <typename T, typename DT>
int sweep_t(cc_ctx *c, T *x, T *f, T *y, T *yp, const T *g, const DT *d, int nsweeps) {
    for (int s = 0; s < nsweeps; ++s) {
        int rc = sweep_rounds_t<T>(c, x, y, g, 0, c->nrounds);
        if (rc) return rc;
        rc = launch_pair_pass<T>(num_pairs(c->n), x, f, yp, g, d, c->stream);
        if (rc) return rc;
    }
    return CC_OK;
}

// tile sizes with a dataflow kernel (the round-by-round executor takes any b)
bool dataflow_b(int b) { return b == 8 || b == 16 || b == 24 || b == 32; }

// workgroups of a dataflow sweep (tables built)
int df_grid(const cc_ctx *c, bool dense) {
    if (c->df_grid_fixed > 0) return std::min(c->df_grid_fixed, c->df_grid_cap);
    return dense ? c->df_grid_dense : c->df_grid_sparse;
}

int ensure_dataflow(cc_ctx *c) {
    if (c->d_dtiles) return CC_OK;
    if (!dataflow_b(c->b)) return fail(CC_EINVAL, "the dataflow executor supports b = 8, 16, 24 and 32");
    std::vector<DTile> tiles;
    std::vector<uint32_t> needs, K;
    try {
        build_dataflow_tables(c->n, c->b, tiles, needs, K);
    } catch (const std::bad_alloc &) {
        return fail(CC_ENOMEM, "no host memory for the dataflow tables");
    }
    c->nblocks = int64_t(K.size());
    c->kmax = 1;
    for (uint32_t v : K) c->kmax = std::max(c->kmax, v);
    if (hipMalloc(&c->d_dtiles, tiles.size() * sizeof(DTile)) != hipSuccess ||
        hipMalloc(&c->d_needs, needs.size() * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->d_K, K.size() * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->d_cnt, K.size() * kCntStride * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->d_ctl, 4 * sizeof(uint32_t)) != hipSuccess)
        return fail(CC_ENOMEM, "hipMalloc of dataflow tables failed");
    CCP_HIP_CHECK(hipMemcpy(c->d_dtiles, tiles.data(), tiles.size() * sizeof(DTile), hipMemcpyHostToDevice));
    CCP_HIP_CHECK(hipMemcpy(c->d_needs, needs.data(), needs.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    CCP_HIP_CHECK(hipMemcpy(c->d_K, K.data(), K.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    int rc = launch_fill_u32(c->nblocks * kCntStride, c->d_cnt, c->stream);
    if (rc) return rc;
    if ((rc = launch_fill_u32(4, c->d_ctl, c->stream))) return rc;
    c->epoch = 0;
    int per_cu = 0, dev = 0, cus = 0, khz = 0;
    rc = (c->prec == CC_F64) ? dataflow_occupancy<double>(c->b, &per_cu) : dataflow_occupancy<float>(c->b, &per_cu);
    if (rc) return rc;
    CCP_HIP_CHECK(hipGetDevice(&dev));
    CCP_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CCP_HIP_CHECK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (per_cu < 1) return fail(CC_EHIP, "dataflow kernel does not fit on a compute unit");
    // Workgroups beyond the schedule's average parallelism only wait, and
    // their polls slow the handoffs on the critical path: at most about
    // (total tile steps) / (critical path) = nb(nb+1)(nb+2)/6 / (4 nb) are
    // useful at once.
    const int64_t nbl = c->nb;
    const int64_t useful = std::max<int64_t>(1, (nbl + 1) * (nbl + 2) / 24);
    const int64_t need_per_cu = std::max<int64_t>(1, (useful + cus - 1) / cus);
    // The sparse and compacted sweeps wait on load latency and gain from
    // every resident workgroup up to that bound.  The dense sweep streams
    // every dual, and more workgroups per CU than these (measured on
    // MI355X over n = 500..4000) contend for HBM and L2 and run slower:
    // b = 8: 4; b = 16: 2 in FP32, 1 in FP64; b = 24, 32: 1.
    const int dense_per_cu = c->b == 8 ? 4 : (c->b == 16 ? (c->prec == CC_F64 ? 1 : 2) : 1);
    c->df_grid_sparse = int(std::min<int64_t>(c->ntiles, std::min<int64_t>(per_cu, need_per_cu) * cus));
    c->df_grid_dense = int(std::min<int64_t>(
        c->ntiles, std::min<int64_t>(std::min<int64_t>(per_cu, need_per_cu), dense_per_cu) * cus));
    c->df_grid_cap = int(std::min<int64_t>(c->ntiles, int64_t(per_cu) * cus));
    c->df_grid_fixed = 0;
    rc = (c->prec == CC_F64) ? aty_dataflow_occupancy<double>(c->b, &per_cu)
                             : aty_dataflow_occupancy<float>(c->b, &per_cu);
    if (rc) return rc;
    if (per_cu < 1) return fail(CC_EHIP, "dataflow A'y kernel does not fit on a compute unit");
    c->aty_grid = int(std::min<int64_t>(c->ntiles, std::min<int64_t>(per_cu, need_per_cu) * cus));
    rc = (c->prec == CC_F64) ? infer_aty_occupancy<double>(c->b, &per_cu) : infer_aty_occupancy<float>(c->b, &per_cu);
    if (rc) return rc;
    if (per_cu < 1) return fail(CC_EHIP, "fused inference kernel does not fit on a compute unit");
    c->iad_grid = int(std::min<int64_t>(c->ntiles, std::min<int64_t>(per_cu, need_per_cu) * cus));
    c->wait_ticks = uint64_t(khz > 0 ? khz : 100000) * 1000ull * 10ull;  // 10 s per wait
    return CC_OK;
}

// mask != nullptr: the sparse dataflow sweep (exec must be CC_EXEC_DATAFLOW)
template <typename T>
int sweep_metric_t(cc_ctx *c, T *x, T *y, const T *g, int exec, unsigned long long *prof,
                   void *mask = nullptr);

template <typename T, typename DT>
int sweep_dataflow_t(cc_ctx *c, T *x, T *f, T *y, T *yp, const T *g, const DT *d,
                     int nsweeps, void *mask = nullptr) {
    int rc;
    for (int s = 0; s < nsweeps; ++s) {
        if ((rc = sweep_metric_t<T>(c, x, y, g, CC_EXEC_DATAFLOW, nullptr, mask))) return rc;
        if ((rc = launch_pair_pass<T>(num_pairs(c->n), x, f, yp, g, d, c->stream))) return rc;
    }
    return CC_OK;
}

// Reports (and clears) an aborted dataflow sweep.  Synchronises.
int check_dataflow(cc_ctx *c) {
    if (!c->d_ctl) return CC_OK;
    uint32_t ctl[4];
    CCP_HIP_CHECK(hipMemcpyAsync(ctl, c->d_ctl, sizeof(ctl), hipMemcpyDeviceToHost, c->stream));
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    if (ctl[1]) {
        // a wait timed out: the state is incomplete; reset the counters
        (void)launch_fill_u32(c->nblocks * kCntStride, c->d_cnt, c->stream);
        (void)launch_fill_u32(4, c->d_ctl, c->stream);
        c->epoch = 0;
        return fail(CC_EHIP, "dataflow sweep aborted: a dependency wait timed out");
    }
    return CC_OK;
}

// Arguments of the next dataflow launch (each launch is one epoch of the
// per-block touch counters).
int dataflow_args(cc_ctx *c, unsigned long long *prof, DataflowArgs &a) {
    int rc = ensure_dataflow(c);
    if (rc) return rc;
    if (uint64_t(c->epoch + 1) * c->kmax >= (1ull << 31)) {
        if ((rc = launch_fill_u32(c->nblocks * kCntStride, c->d_cnt, c->stream))) return rc;
        c->epoch = 0;
    }
    a = DataflowArgs{c->d_dtiles, int(c->ntiles), c->d_needs, c->d_K, c->d_cnt, c->d_ctl,
                     c->epoch, c->wait_ticks, prof};
    return CC_OK;
}

// The FP64 dense dataflow sweep (like the sparse one) addresses a tile's
// duals, at most ceil(n/b) steps of 3 b^3, with 31-bit byte offsets.
int check_tile_offsets(const cc_ctx *c) {
    if (c->prec == CC_F64 && int64_t(c->nb) * 3 * c->b * c->b * c->b * int64_t(elem_size(c)) >= (int64_t(1) << 31))
        return fail(CC_EINVAL, "the FP64 dataflow sweep addresses a tile's duals with 31-bit offsets: n too large for b");
    return CC_OK;
}

template <typename T>
int sweep_metric_t(cc_ctx *c, T *x, T *y, const T *g, int exec, unsigned long long *prof,
                   void *mask) {
    if (exec == CC_EXEC_ROUNDS) return sweep_rounds_t<T>(c, x, y, g, 0, c->nrounds);
    int rc = check_tile_offsets(c);
    if (rc) return rc;
    DataflowArgs a;
    rc = dataflow_args(c, prof, a);
    if (rc) return rc;
    if ((rc = launch_sweep_dataflow<T>(a, df_grid(c, mask == nullptr), c->b, c->n, x, g, y, mask, nullptr,
                                       c->stream)))
        return rc;
    c->epoch++;
    return CC_OK;
}

// The dataflow sweep over the tiles of the first `rounds` rounds only.
// Tickets run in schedule order, and a tile of round r waits only on
// touches by tiles of rounds <= r, so the prefix needs nothing beyond it.
// The counters then hold a partial epoch and are cleared.
template <typename T>
int sweep_prefix_t(cc_ctx *c, T *x, T *y, const T *g, int rounds) {
    int rc = check_tile_offsets(c);
    if (rc) return rc;
    DataflowArgs a;
    rc = dataflow_args(c, nullptr, a);
    if (rc) return rc;
    a.ntiles = int(c->round_start[rounds]);
    if (a.ntiles > 0 &&
        (rc = launch_sweep_dataflow<T>(a, df_grid(c, true), c->b, c->n, x, g, y, nullptr, nullptr, c->stream)))
        return rc;
    if ((rc = launch_fill_u32(c->nblocks * kCntStride, c->d_cnt, c->stream))) return rc;
    c->epoch = 0;
    return check_dataflow(c);
}

int ensure_ax(cc_ctx *c) {
    if (!c->d_ax) {
        if (hipMalloc(&c->d_ax, size_t(num_pairs(c->n)) * sizeof(double)) != hipSuccess) {
            c->d_ax = nullptr;
            return fail(CC_ENOMEM, "hipMalloc of the A'y accumulator failed");
        }
    }
    return CC_OK;
}

template <typename T>
int aty_t(cc_ctx *c, const T *y) {
    int rc = ensure_ax(c);
    if (rc) return rc;
    CCP_HIP_CHECK(hipMemsetAsync(c->d_ax, 0, size_t(num_pairs(c->n)) * sizeof(double), c->stream));
    if (dataflow_b(c->b)) {
        DataflowArgs a;
        if ((rc = dataflow_args(c, nullptr, a))) return rc;
        if ((rc = launch_aty_dataflow<T>(a, c->aty_grid, c->b, c->n, y, c->d_ax, c->stream))) return rc;
        c->epoch++;
        return CC_OK;
    }
    for (int r = 0; r < c->nrounds; ++r) {
        const int64_t a = c->round_start[r], e = c->round_start[r + 1];
        rc = launch_aty_round<T>(c->d_tiles + a, int(e - a), c->b, c->n, y, c->d_ax, c->stream);
        if (rc) return rc;
    }
    return CC_OK;
}

template <typename T, typename DT>
int residuals_t(cc_ctx *c, const T *x, const T *f, const T *y, const T *yp, const double *w,
                const DT *d, double gamma, int what, cc_resid *out) {
    const bool want_cs = (what & CC_RESID_CS) && y;
    const bool want_dual = (what & CC_RESID_DUAL) && y && yp;
    int rc;
    if (want_dual) {
        rc = aty_t<T>(c, y);
        if (rc) return rc;
    }
    rc = launch_metric_resid<T>(c->d_tiles, c->d_chunks, c->nchunks, c->b, c->n, x, want_cs ? y : nullptr,
                                c->d_mpart, c->stream);
    if (rc) return rc;
    rc = launch_pair_resid<T>(num_pairs(c->n), x, f, (want_cs || want_dual) ? yp : nullptr, w, d,
                              want_dual ? c->d_ax : nullptr, gamma, c->d_ppart, c->stream);
    if (rc) return rc;
    rc = launch_final_reduce(c->d_mpart, c->nchunks, c->d_ppart, c->d_out, c->stream);
    if (rc) return rc;
    double h[14];
    CCP_HIP_CHECK(hipMemcpyAsync(h, c->d_out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    if (want_dual && (rc = check_dataflow(c))) return rc;
    const double nan = std::nan("");
    // h: 0 metric max viol, 1 metric cs sum, 2 metric cs max, 3 metric bad,
    //    4 pair max viol, 5 sum w f, 6 sum w (x^2+f^2), 7 lp, 8 pair cs max,
    //    9 pair cs sum, 10 quad dual, 11 b'y, 12 stat, 13 pair bad
    out->max_viol_metric = h[0];
    out->max_viol_pair = h[4];
    out->primal_qp = h[5] + h[6] / (2.0 * gamma);
    out->lp_cost = h[7];
    out->cs_max = want_cs ? std::fmax(h[2], h[8]) : nan;
    if (want_dual) {
        out->dual_qp = -h[11] - 0.5 * gamma * h[10];
        out->gap = out->primal_qp - out->dual_qp;
        out->stat_resid = h[12];
    } else {
        out->dual_qp = out->gap = out->stat_resid = nan;
    }
    if (h[3] != 0.0 || h[13] != 0.0 || !std::isfinite(out->primal_qp))
        return fail(CC_ENONFINITE, "non-finite value in x or f");
    return CC_OK;
}

// l2 metric nearness: the metric rows' residuals as for (qp), the pair terms
// from k_nearness_pair_resid in k_pair_resid's slots.
template <typename T>
int nearness_residuals_t(cc_ctx *c, const T *x, const T *y, const double *w, const double *dv, int what,
                         cc_nresid *out) {
    const bool want_cs = (what & CC_RESID_CS) && y;
    const bool want_dual = (what & CC_RESID_DUAL) && y;
    int rc;
    if (want_dual && (rc = aty_t<T>(c, y))) return rc;
    rc = launch_metric_resid<T>(c->d_tiles, c->d_chunks, c->nchunks, c->b, c->n, x, want_cs ? y : nullptr,
                                c->d_mpart, c->stream);
    if (rc) return rc;
    rc = launch_nearness_pair_resid<T>(num_pairs(c->n), x, dv, w, want_dual ? c->d_ax : nullptr,
                                       c->d_ppart, c->stream);
    if (rc) return rc;
    if ((rc = launch_final_reduce(c->d_mpart, c->nchunks, c->d_ppart, c->d_out, c->stream))) return rc;
    double h[14];
    CCP_HIP_CHECK(hipMemcpyAsync(h, c->d_out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    if (want_dual && (rc = check_dataflow(c))) return rc;
    const double nan = std::nan("");
    // h: 0 metric max viol, 2 metric cs max, 3 metric bad, 6 sum w (x-d)^2,
    //    10 sum (A'y)^2 / w, 11 d'A'y, 12 stationarity, 13 pair bad
    out->max_viol = h[0];
    out->primal = 0.5 * h[6];
    out->cs_max = want_cs ? h[2] : nan;
    if (want_dual) {
        out->dual = h[11] - 0.5 * h[10];
        out->gap = out->primal - out->dual;
        out->stat_resid = h[12];
    } else {
        out->dual = out->gap = out->stat_resid = nan;
    }
    if (h[3] != 0.0 || h[13] != 0.0 || !std::isfinite(out->primal))
        return fail(CC_ENONFINITE, "non-finite value in x");
    return CC_OK;
}

template <typename T>
int x_from_y_t(cc_ctx *c, const T *y, const T *yp, const double *w, double gamma, T *x, T *f) {
    int rc = aty_t<T>(c, y);
    if (rc) return rc;
    return launch_x_from_aty<T>(num_pairs(c->n), c->d_ax, yp, w, gamma, x, f, c->stream);
}

}  // namespace

extern "C" {

const char *cc_last_error(void) { return g_last_error.c_str(); }

int64_t cc_num_metric_duals(int64_t n) {
    if (n < 3) return 0;
    return 3 * (n * (n - 1) * (n - 2) / 6);
}

int cc_create(cc_ctx **out, int64_t n, int32_t b, int32_t prec, void *stream) {
    if (!out) return fail(CC_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 3) return fail(CC_EINVAL, "n must be at least 3");
    if (n > (int64_t(1) << 20)) return fail(CC_EINVAL, "n too large");
    if (b < 1 || b > 32) return fail(CC_EINVAL, "tile size b must be in 1..32");
    if (prec != CC_F64 && prec != CC_F32) return fail(CC_EINVAL, "prec must be CC_F64 or CC_F32");
    cc_ctx *c = new (std::nothrow) cc_ctx();
    if (!c) return fail(CC_ENOMEM, "context allocation failed");
    c->n = n;
    c->b = b;
    c->prec = prec;
    c->stream = static_cast<hipStream_t>(stream);
    c->nb = int((n + b - 1) / b);
    c->nrounds = 2 * c->nb - 1;
    std::vector<Tile> tiles;
    std::vector<int32_t> chunks;
    try {
        build_schedule(c, tiles);
        for (size_t t = 0; t < tiles.size(); ++t)
            for (int m0 = 0; m0 <= tiles[t].Q - tiles[t].P; m0 += kChunkSteps) {
                chunks.push_back(int32_t(t));
                chunks.push_back(m0);
            }
    } catch (const std::bad_alloc &) {
        cc_destroy(c);
        return fail(CC_ENOMEM, "no host memory for the schedule");
    }
    c->nchunks = int64_t(chunks.size() / 2);
    int rc = CC_OK;
    if (hipMalloc(&c->d_tiles, tiles.size() * sizeof(Tile)) != hipSuccess ||
        hipMalloc(&c->d_chunks, chunks.size() * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c->d_mpart, size_t(c->nchunks) * 4 * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_ppart, size_t(pair_partial_blocks()) * 10 * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_out, 16 * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_flag, sizeof(int)) != hipSuccess) {
        cc_destroy(c);
        return fail(CC_ENOMEM, "hipMalloc of schedule tables failed");
    }
    if (hipMemcpy(c->d_tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c->d_chunks, chunks.data(), chunks.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
            hipSuccess) {
        cc_destroy(c);
        return fail(CC_EHIP, "copy of schedule tables failed");
    }
    rc = (prec == CC_F64) ? set_sweep_lds_limits<double>(b) : set_sweep_lds_limits<float>(b);
    // the dataflow executor's tables, built here so that no later sweep
    // allocates (cc_sweep_noalloc relies on it)
    if (!rc && dataflow_b(b)) rc = ensure_dataflow(c);
    if (rc) {
        cc_destroy(c);
        return rc;
    }
    *out = c;
    return CC_OK;
}

static void compact_free(cc_ctx *c) {
    for (int e = 0; e < 2; ++e) {
        (void)hipFree(c->cp_idx[e]);
        (void)hipFree(c->cp_val[e]);
        (void)hipFree(c->cp_off[e]);
        (void)hipFree(c->cp_cnt[e]);
        c->cp_idx[e] = nullptr;
        c->cp_val[e] = nullptr;
        c->cp_off[e] = nullptr;
        c->cp_cnt[e] = nullptr;
        c->cp_cap[e] = 0;
    }
    (void)hipFree(c->cp_alloc);
    (void)hipFree(c->cp_flag);
    (void)hipFree(c->cp_xsnap);
    (void)hipFree(c->cp_step_tile);
    c->cp_alloc = nullptr;
    c->cp_flag = nullptr;
    c->cp_xsnap = nullptr;
    c->cp_step_tile = nullptr;
    c->cp_nnz = 0;
    c->cp_regrows = 0;
}

int cc_destroy(cc_ctx *c) {
    if (!c) return CC_OK;
    compact_free(c);
    (void)hipFree(c->d_tiles);
    (void)hipFree(c->d_mpart);
    (void)hipFree(c->d_ppart);
    (void)hipFree(c->d_out);
    (void)hipFree(c->d_flag);
    (void)hipFree(c->d_ax);
    (void)hipFree(c->d_dtiles);
    (void)hipFree(c->d_needs);
    (void)hipFree(c->d_K);
    (void)hipFree(c->d_cnt);
    (void)hipFree(c->d_ctl);
    (void)hipFree(c->d_mean_deg);
    (void)hipFree(c->d_chunks);
    delete c;
    return CC_OK;
}

int64_t cc_dual_slots(const cc_ctx *c) { return c ? c->slots : 0; }
int32_t cc_num_rounds(const cc_ctx *c) { return c ? c->nrounds : 0; }

int cc_prepare(cc_ctx *c, const double *w, double gamma, void *g) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(w, "w")) || (rc = need(g, "g"))) return rc;
    if (!(gamma > 0.0) || !std::isfinite(gamma)) return fail(CC_EINVAL, "gamma must be finite and > 0");
    CCP_HIP_CHECK(hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
    const int64_t np = num_pairs(c->n);
    rc = (c->prec == CC_F64)
             ? launch_prepare<double>(np, w, gamma, static_cast<double *>(g), c->d_flag, c->stream)
             : launch_prepare<float>(np, w, gamma, static_cast<float *>(g), c->d_flag, c->stream);
    if (rc) return rc;
    int bad = 0;
    CCP_HIP_CHECK(hipMemcpyAsync(&bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    if (bad) return fail(CC_EINVAL, "every weight must be finite and > 0");
    return CC_OK;
}

int cc_init_cold(cc_ctx *c, void *x, void *f, void *y, void *yp, double gamma) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(f, "f")) || (rc = need(yp, "y_pair")))
        return rc;
    if (!(gamma > 0.0) || !std::isfinite(gamma)) return fail(CC_EINVAL, "gamma must be finite and > 0");
    const int64_t np = num_pairs(c->n);
    if (c->prec == CC_F64)
        return launch_init_cold<double>(np, c->slots, (double *)x, (double *)f, (double *)y,
                                        (double *)yp, gamma, c->stream);
    return launch_init_cold<float>(np, c->slots, (float *)x, (float *)f, (float *)y, (float *)yp,
                                   gamma, c->stream);
}

int cc_sweep(cc_ctx *c, void *x, void *f, void *y, void *yp, const void *g, const uint8_t *d,
             int32_t nsweeps, int32_t exec) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(f, "f")) || (rc = need(y, "y")) ||
        (rc = need(yp, "y_pair")) || (rc = need(g, "g")) || (rc = need(d, "d")))
        return rc;
    if (nsweeps < 0) return fail(CC_EINVAL, "nsweeps must be >= 0");
    if (exec != CC_EXEC_ROUNDS && exec != CC_EXEC_DATAFLOW) return fail(CC_EINVAL, "unknown executor");
    if (exec == CC_EXEC_DATAFLOW) {
        if (c->prec == CC_F64)
            return sweep_dataflow_t<double>(c, (double *)x, (double *)f, (double *)y, (double *)yp,
                                            (const double *)g, d, nsweeps);
        return sweep_dataflow_t<float>(c, (float *)x, (float *)f, (float *)y, (float *)yp,
                                       (const float *)g, d, nsweeps);
    }
    if (c->prec == CC_F64)
        return sweep_t<double>(c, (double *)x, (double *)f, (double *)y, (double *)yp,
                               (const double *)g, d, nsweeps);
    return sweep_t<float>(c, (float *)x, (float *)f, (float *)y, (float *)yp, (const float *)g, d,
                          nsweeps);
}

}  // extern "C"

// ----- allocation-free sweeps ----------------------------------------------
// The dataflow executor's scratch (ticket counter, abort flag and one touch
// counter per block of x) in a static device array instead of the context's
// buffers: no allocation at all per call.  Each device holds its own copy;
// its address is taken once per device (hipGetSymbolAddress) and only that
// address reaches the kernels (the array's name in host code is a host-side
// stand-in, not a device address).  Layout: words [0, 64) control ([0]
// ticket, [1] abort flag), then kCntStride words per block.

constexpr int64_t kNoallocScratchBytes = int64_t(4) << 20;
constexpr int64_t kNoallocCtlWords = 64;
constexpr int64_t kNoallocMaxBlocks =
    (kNoallocScratchBytes / int64_t(sizeof(uint32_t)) - kNoallocCtlWords) / kCntStride;
static __device__ __align__(256) uint32_t scratch[kNoallocScratchBytes / sizeof(uint32_t)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch` (set-up on the
// first call on each device, with that device current).
int scratch_address(uint32_t **out) {
    int dev = 0;
    CCP_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CC_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<uint32_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return CC_OK;
}

template <typename T>
int sweep_noalloc_t(cc_ctx *c, uint32_t *ws, T *x, T *f, T *y, T *yp, const T *g, const uint8_t *d,
                    int nsweeps) {
    uint32_t *const ctl = ws, *const cnt = ws + kNoallocCtlWords;
    int rc = check_tile_offsets(c);
    if (rc) return rc;
    // every call starts from zeroed counters and flags (a fill kernel)
    if ((rc = launch_fill_u32(kNoallocCtlWords + c->nblocks * kCntStride, ws, c->stream))) return rc;
    for (int s = 0; s < nsweeps; ++s) {
        const DataflowArgs a{c->d_dtiles, int(c->ntiles), c->d_needs, c->d_K, cnt, ctl,
                             uint32_t(s), c->wait_ticks, nullptr};
        if ((rc = launch_sweep_dataflow<T>(a, df_grid(c, true), c->b, c->n, x, g, y, nullptr, nullptr,
                                           c->stream)))
            return rc;
        if ((rc = launch_pair_pass<T>(num_pairs(c->n), x, f, yp, g, d, c->stream))) return rc;
    }
    uint32_t h[2] = {0u, 0u};
    CCP_HIP_CHECK(hipMemcpyAsync(h, ctl, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    if (h[1]) return fail(CC_EHIP, "dataflow sweep aborted: a dependency wait timed out");
    return CC_OK;
}
}  // namespace

extern "C" {

int cc_sweep_noalloc(cc_ctx *c, void *x, void *f, void *y, void *yp, const void *g, const uint8_t *d,
                     int32_t nsweeps) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(f, "f")) || (rc = need(y, "y")) ||
        (rc = need(yp, "y_pair")) || (rc = need(g, "g")) || (rc = need(d, "d")))
        return rc;
    if (nsweeps < 0) return fail(CC_EINVAL, "nsweeps must be >= 0");
    if (!dataflow_b(c->b) || !c->d_dtiles)
        return fail(CC_EINVAL, "cc_sweep_noalloc needs the dataflow executor (b = 8, 16, 24, 32)");
    if (c->nblocks > kNoallocMaxBlocks)
        return fail(CC_EINVAL, "cc_sweep_noalloc: " + std::to_string(c->nblocks) +
                                   " blocks of x exceed its static scratch (" +
                                   std::to_string(kNoallocMaxBlocks) + " blocks: ceil(n/b) <= 255)");
    if ((int64_t(nsweeps) + 1) * c->kmax >= (int64_t(1) << 31))
        return fail(CC_EINVAL, "cc_sweep_noalloc: too many sweeps in one call");
    uint32_t *ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    if (c->prec == CC_F64)
        return sweep_noalloc_t<double>(c, ws, (double *)x, (double *)f, (double *)y, (double *)yp,
                                       (const double *)g, d, nsweeps);
    return sweep_noalloc_t<float>(c, ws, (float *)x, (float *)f, (float *)y, (float *)yp,
                                  (const float *)g, d, nsweeps);
}

int cc_sweep_metric(cc_ctx *c, void *x, void *y, const void *g, int32_t exec) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(y, "y")) || (rc = need(g, "g")))
        return rc;
    if (exec != CC_EXEC_ROUNDS && exec != CC_EXEC_DATAFLOW) return fail(CC_EINVAL, "unknown executor");
    if (c->prec == CC_F64) return sweep_metric_t<double>(c, (double *)x, (double *)y, (const double *)g, exec, nullptr);
    return sweep_metric_t<float>(c, (float *)x, (float *)y, (const float *)g, exec, nullptr);
}

int64_t cc_dual_mask_bytes(const cc_ctx *c) {
    if (!c || !dataflow_b(c->b)) return -1;
    // one word per b slots: b / 8 bytes, 4 for b = 24
    return c->slots / c->b * (c->b == 24 ? 4 : c->b / 8);
}

int cc_dual_mask_build(cc_ctx *c, const void *y, void *mask) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(y, "y")) || (rc = need(mask, "mask"))) return rc;
    const int64_t nsteps = c->slots / (int64_t(3) * c->b * c->b * c->b);
    if (c->prec == CC_F64) return launch_mask_build<double>(c->b, nsteps, (const double *)y, mask, c->stream);
    return launch_mask_build<float>(c->b, nsteps, (const float *)y, mask, c->stream);
}

int cc_sweep_sparse(cc_ctx *c, void *x, void *f, void *y, void *yp, const void *g, const uint8_t *d,
                    void *mask, int32_t nsweeps) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(f, "f")) || (rc = need(y, "y")) ||
        (rc = need(yp, "y_pair")) || (rc = need(g, "g")) || (rc = need(d, "d")) || (rc = need(mask, "mask")))
        return rc;
    if (nsweeps < 0) return fail(CC_EINVAL, "nsweeps must be >= 0");
    if (!dataflow_b(c->b)) return fail(CC_EINVAL, "sparse sweeps need b = 8, 16, 24 or 32");
    if (int64_t(c->nb) * 3 * c->b * c->b * c->b * int64_t(elem_size(c)) >= (int64_t(1) << 31))
        return fail(CC_EINVAL, "sparse sweeps address a tile's duals with 31-bit offsets: n too large for b");
    if (c->prec == CC_F64)
        return sweep_dataflow_t<double>(c, (double *)x, (double *)f, (double *)y, (double *)yp,
                                        (const double *)g, d, nsweeps, mask);
    return sweep_dataflow_t<float>(c, (float *)x, (float *)f, (float *)y, (float *)yp, (const float *)g,
                                   d, nsweeps, mask);
}

int cc_sweep_metric_sparse(cc_ctx *c, void *x, void *y, const void *g, void *mask) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(y, "y")) || (rc = need(g, "g")) ||
        (rc = need(mask, "mask")))
        return rc;
    if (!dataflow_b(c->b)) return fail(CC_EINVAL, "sparse sweeps need b = 8, 16, 24 or 32");
    if (int64_t(c->nb) * 3 * c->b * c->b * c->b * int64_t(elem_size(c)) >= (int64_t(1) << 31))
        return fail(CC_EINVAL, "sparse sweeps address a tile's duals with 31-bit offsets: n too large for b");
    if (c->prec == CC_F64)
        return sweep_metric_t<double>(c, (double *)x, (double *)y, (const double *)g, CC_EXEC_DATAFLOW, nullptr, mask);
    return sweep_metric_t<float>(c, (float *)x, (float *)y, (const float *)g, CC_EXEC_DATAFLOW, nullptr, mask);
}

int cc_l1_sweep(cc_ctx *c, void *x, void *f, void *y, void *yp, const void *g, const double *dv,
                void *mask, int32_t nsweeps) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(f, "f")) || (rc = need(y, "y")) ||
        (rc = need(yp, "y_pair")) || (rc = need(g, "g")) || (rc = need(dv, "d")))
        return rc;
    if (nsweeps < 0) return fail(CC_EINVAL, "nsweeps must be >= 0");
    const bool df = dataflow_b(c->b);
    if (mask && !df) return fail(CC_EINVAL, "sparse sweeps need b = 8, 16, 24 or 32");
    if (mask && int64_t(c->nb) * 3 * c->b * c->b * c->b * int64_t(elem_size(c)) >= (int64_t(1) << 31))
        return fail(CC_EINVAL, "sparse sweeps address a tile's duals with 31-bit offsets: n too large for b");
    if (c->prec == CC_F64) {
        if (df)
            return sweep_dataflow_t<double>(c, (double *)x, (double *)f, (double *)y, (double *)yp,
                                            (const double *)g, dv, nsweeps, mask);
        return sweep_t<double>(c, (double *)x, (double *)f, (double *)y, (double *)yp, (const double *)g, dv,
                               nsweeps);
    }
    if (df)
        return sweep_dataflow_t<float>(c, (float *)x, (float *)f, (float *)y, (float *)yp, (const float *)g, dv,
                                       nsweeps, mask);
    return sweep_t<float>(c, (float *)x, (float *)f, (float *)y, (float *)yp, (const float *)g, dv, nsweeps);
}

int cc_l1_residuals(cc_ctx *c, const void *x, const void *f, const void *y, const void *yp, const double *w,
                    const double *dv, double gamma, int32_t what, cc_resid *out) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(f, "f")) || (rc = need(w, "w")) ||
        (rc = need(dv, "d")) || (rc = need(out, "out")))
        return rc;
    if (!(gamma > 0.0)) return fail(CC_EINVAL, "gamma must be > 0");
    if (c->prec == CC_F64)
        return residuals_t<double>(c, (const double *)x, (const double *)f, (const double *)y,
                                   (const double *)yp, w, dv, gamma, what, out);
    return residuals_t<float>(c, (const float *)x, (const float *)f, (const float *)y, (const float *)yp, w,
                              dv, gamma, what, out);
}

}  // extern "C"

namespace {

// (Re)allocates pool e with room for cap entries.
int compact_pool(cc_ctx *c, int e, int64_t cap) {
    (void)hipFree(c->cp_idx[e]);
    (void)hipFree(c->cp_val[e]);
    c->cp_idx[e] = nullptr;
    c->cp_val[e] = nullptr;
    c->cp_cap[e] = 0;
    if (hipMalloc(&c->cp_idx[e], size_t(cap) * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&c->cp_val[e], size_t(cap) * elem_size(c)) != hipSuccess)
        return fail(CC_ENOMEM, "hipMalloc of a compacted dual pool failed");
    c->cp_cap[e] = cap;
    return CC_OK;
}

int64_t num_steps(const cc_ctx *c) { return c->slots / (int64_t(3) * c->b * c->b * c->b); }

template <typename T>
int sweep_compact_t(cc_ctx *c, T *x, T *f, T *yp, const T *g, const uint8_t *d, int nsweeps) {
    int rc;
    const int64_t np = num_pairs(c->n);
    for (int s = 0; s < nsweeps; ++s) {
        for (int attempt = 0;; ++attempt) {
            const int in = c->cp_cur, out = 1 - c->cp_cur;
            CCP_HIP_CHECK(hipMemcpyAsync(c->cp_xsnap, x, size_t(np) * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
            CCP_HIP_CHECK(hipMemsetAsync(c->cp_alloc, 0, sizeof(unsigned long long), c->stream));
            CCP_HIP_CHECK(hipMemsetAsync(c->cp_flag, 0, sizeof(uint32_t), c->stream));
            DataflowArgs a;
            if ((rc = dataflow_args(c, nullptr, a))) return rc;
            const CompactArgs<T> ca{c->cp_idx[in], static_cast<const T *>(c->cp_val[in]), c->cp_off[in],
                                    c->cp_cnt[in], c->cp_idx[out], static_cast<T *>(c->cp_val[out]),
                                    c->cp_off[out], c->cp_cnt[out], c->cp_alloc, c->cp_cap[out], c->cp_flag};
            if ((rc = launch_sweep_dataflow<T>(a, df_grid(c, false), c->b, c->n, x, g, nullptr, nullptr, &ca,
                                               c->stream)))
                return rc;
            c->epoch++;
            if ((rc = check_dataflow(c))) return rc;
            unsigned long long used = 0;
            uint32_t flag = 0;
            CCP_HIP_CHECK(hipMemcpyAsync(&used, c->cp_alloc, sizeof(used), hipMemcpyDeviceToHost, c->stream));
            CCP_HIP_CHECK(hipMemcpyAsync(&flag, c->cp_flag, sizeof(flag), hipMemcpyDeviceToHost, c->stream));
            CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
            if (!flag) {
                c->cp_nnz = int64_t(used);
                c->cp_cur = out;
                break;
            }
            // the new lists did not fit: the input lists are intact, so
            // restore x and repeat the sweep into a larger pool
            if (attempt >= 4) return fail(CC_ENOMEM, "compacted dual pool kept overflowing");
            CCP_HIP_CHECK(hipMemcpyAsync(x, c->cp_xsnap, size_t(np) * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
            const int64_t want = int64_t(used) + int64_t(used) / 4 + 4096;
            if ((rc = compact_pool(c, out, std::max<int64_t>(want, 2 * c->cp_cap[out])))) return rc;
            c->cp_regrows++;
        }
        if ((rc = launch_pair_pass<T>(np, x, f, yp, g, d, c->stream))) return rc;
    }
    return CC_OK;
}

}  // namespace

extern "C" {

int cc_compact_init(cc_ctx *c, int64_t capacity) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if (!(c->b == 8 || c->b == 16)) return fail(CC_EINVAL, "compacted dual lists need b = 8 or 16");
    if (capacity < 1) return fail(CC_EINVAL, "capacity must be >= 1");
    if ((rc = ensure_dataflow(c))) return rc;
    compact_free(c);
    const int64_t ns = num_steps(c);
    for (int e = 0; e < 2; ++e) {
        if (hipMalloc(&c->cp_off[e], size_t(ns) * sizeof(int64_t)) != hipSuccess ||
            hipMalloc(&c->cp_cnt[e], size_t(ns) * sizeof(uint32_t)) != hipSuccess) {
            compact_free(c);
            return fail(CC_ENOMEM, "hipMalloc of compacted list tables failed");
        }
        if ((rc = compact_pool(c, e, capacity))) {
            compact_free(c);
            return rc;
        }
    }
    if (hipMalloc(&c->cp_alloc, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->cp_flag, sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->cp_xsnap, size_t(num_pairs(c->n)) * elem_size(c)) != hipSuccess ||
        hipMalloc(&c->cp_step_tile, size_t(ns) * sizeof(int32_t)) != hipSuccess) {
        compact_free(c);
        return fail(CC_ENOMEM, "hipMalloc for compacted lists failed");
    }
    // tile of every step, for export
    std::vector<DTile> tiles;
    std::vector<uint32_t> needs, K;
    std::vector<int32_t> st;
    try {
        build_dataflow_tables(c->n, c->b, tiles, needs, K);
        st.assign(size_t(ns), 0);
    } catch (const std::bad_alloc &) {
        compact_free(c);
        return fail(CC_ENOMEM, "no host memory for the step table");
    }
    for (size_t t = 0; t < tiles.size(); ++t)
        for (int m = 0; m <= tiles[t].Q - tiles[t].P; ++m) st[size_t(tiles[t].jsbase) + m] = int32_t(t);
    CCP_HIP_CHECK(hipMemcpy(c->cp_step_tile, st.data(), st.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    // the cold start: every list empty
    CCP_HIP_CHECK(hipMemsetAsync(c->cp_cnt[0], 0, size_t(ns) * sizeof(uint32_t), c->stream));
    CCP_HIP_CHECK(hipMemsetAsync(c->cp_off[0], 0, size_t(ns) * sizeof(int64_t), c->stream));
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    c->cp_cur = 0;
    c->cp_nnz = 0;
    return CC_OK;
}

int cc_sweep_compact(cc_ctx *c, void *x, void *f, void *yp, const void *g, const uint8_t *d, int32_t nsweeps) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(f, "f")) || (rc = need(yp, "y_pair")) ||
        (rc = need(g, "g")) || (rc = need(d, "d")))
        return rc;
    if (!c->cp_cnt[0]) return fail(CC_EINVAL, "call cc_compact_init first");
    if (nsweeps < 0) return fail(CC_EINVAL, "nsweeps must be >= 0");
    if (c->prec == CC_F64)
        return sweep_compact_t<double>(c, (double *)x, (double *)f, (double *)yp, (const double *)g, d, nsweeps);
    return sweep_compact_t<float>(c, (float *)x, (float *)f, (float *)yp, (const float *)g, d, nsweeps);
}

int cc_compact_to_slots(cc_ctx *c, void *y) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(y, "y"))) return rc;
    if (!c->cp_cnt[0]) return fail(CC_EINVAL, "call cc_compact_init first");
    const int in = c->cp_cur;
    CCP_HIP_CHECK(hipMemsetAsync(y, 0, size_t(c->slots) * elem_size(c), c->stream));
    if (c->prec == CC_F64)
        return launch_compact_to_slots<double>(c->b, num_steps(c), c->cp_idx[in], (const double *)c->cp_val[in],
                                               c->cp_off[in], c->cp_cnt[in], (double *)y, c->stream);
    return launch_compact_to_slots<float>(c->b, num_steps(c), c->cp_idx[in], (const float *)c->cp_val[in],
                                          c->cp_off[in], c->cp_cnt[in], (float *)y, c->stream);
}

int cc_compact_export(cc_ctx *c, int64_t *lex, void *val, int64_t capacity, int64_t *count) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(count, "count"))) return rc;
    if (!c->cp_cnt[0]) return fail(CC_EINVAL, "call cc_compact_init first");
    *count = c->cp_nnz;
    if (!lex || !val || capacity < c->cp_nnz) return CC_OK;
    const int in = c->cp_cur;
    if (c->prec == CC_F64)
        rc = launch_compact_export<double>(c->b, num_steps(c), c->nb, c->d_dtiles, c->cp_step_tile, c->cp_idx[in],
                                           (const double *)c->cp_val[in], c->cp_off[in], c->cp_cnt[in], lex,
                                           (double *)val, c->stream);
    else
        rc = launch_compact_export<float>(c->b, num_steps(c), c->nb, c->d_dtiles, c->cp_step_tile, c->cp_idx[in],
                                          (const float *)c->cp_val[in], c->cp_off[in], c->cp_cnt[in], lex,
                                          (float *)val, c->stream);
    if (rc) return rc;
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    return CC_OK;
}

int cc_compact_info(cc_ctx *c, int64_t *nnz, int64_t *bytes, int32_t *regrows) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    int64_t by = 0;
    if (c->cp_cnt[0]) {
        by = (c->cp_cap[0] + c->cp_cap[1]) * int64_t(sizeof(uint16_t) + elem_size(c)) +
             2 * num_steps(c) * int64_t(sizeof(int64_t) + sizeof(uint32_t)) + num_steps(c) * int64_t(sizeof(int32_t)) +
             num_pairs(c->n) * int64_t(elem_size(c));
    }
    if (nnz) *nnz = c->cp_nnz;
    if (bytes) *bytes = by;
    if (regrows) *regrows = c->cp_regrows;
    return CC_OK;
}

int cc_compact_release(cc_ctx *c) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    compact_free(c);
    return CC_OK;
}

int cc_init_cold_lex(cc_ctx *c, void *x, void *f, void *y_lex, void *yp, double gamma) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(f, "f")) || (rc = need(y_lex, "y_lex")) ||
        (rc = need(yp, "y_pair")))
        return rc;
    if (!(gamma > 0.0) || !std::isfinite(gamma)) return fail(CC_EINVAL, "gamma must be finite and > 0");
    const int64_t np = num_pairs(c->n), nm = cc_num_metric_duals(c->n);
    if (c->prec == CC_F64)
        return launch_init_cold<double>(np, nm, (double *)x, (double *)f, (double *)y_lex, (double *)yp, gamma,
                                        c->stream);
    return launch_init_cold<float>(np, nm, (float *)x, (float *)f, (float *)y_lex, (float *)yp, gamma, c->stream);
}

int cc_sweep_colour(cc_ctx *c, void *x, void *f, void *y_lex, void *yp, const void *g, const uint8_t *d,
                    int32_t nsweeps) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(f, "f")) || (rc = need(y_lex, "y_lex")) ||
        (rc = need(yp, "y_pair")) || (rc = need(g, "g")) || (rc = need(d, "d")))
        return rc;
    if (nsweeps < 0) return fail(CC_EINVAL, "nsweeps must be >= 0");
    const int64_t np = num_pairs(c->n);
    for (int s = 0; s < nsweeps; ++s) {
        if (c->prec == CC_F64) {
            if ((rc = launch_sweep_colour<double>(c->n, (double *)x, (const double *)g, (double *)y_lex, c->stream)) ||
                (rc = launch_pair_pass<double>(np, (double *)x, (double *)f, (double *)yp, (const double *)g, d,
                                               c->stream)))
                return rc;
        } else {
            if ((rc = launch_sweep_colour<float>(c->n, (float *)x, (const float *)g, (float *)y_lex, c->stream)) ||
                (rc = launch_pair_pass<float>(np, (float *)x, (float *)f, (float *)yp, (const float *)g, d,
                                              c->stream)))
                return rc;
        }
    }
    return CC_OK;
}

int cc_set_dataflow_workgroups(cc_ctx *c, int32_t workgroups, int32_t *effective) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if (workgroups < 0) return fail(CC_EINVAL, "workgroups must be >= 0");
    if ((rc = ensure_dataflow(c))) return rc;
    c->df_grid_fixed = workgroups;
    if (effective) *effective = df_grid(c, true);
    return CC_OK;
}

int cc_dataflow_breakdown(cc_ctx *c, void *x, void *y, const void *g, double *out) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(y, "y")) || (rc = need(g, "g")) ||
        (rc = need(out, "out")))
        return rc;
    DevTmp t;
    if ((rc = t.alloc(8 * sizeof(unsigned long long)))) return rc;
    CCP_HIP_CHECK(hipMemsetAsync(t.p, 0, 8 * sizeof(unsigned long long), c->stream));
    unsigned long long *prof = (unsigned long long *)t.p;
    rc = (c->prec == CC_F64)
             ? sweep_metric_t<double>(c, (double *)x, (double *)y, (const double *)g, CC_EXEC_DATAFLOW, prof)
             : sweep_metric_t<float>(c, (float *)x, (float *)y, (const float *)g, CC_EXEC_DATAFLOW, prof);
    if (rc) return rc;
    unsigned long long h[8];
    CCP_HIP_CHECK(hipMemcpyAsync(h, prof, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    if ((rc = check_dataflow(c))) return rc;
    int dev = 0, khz = 0;
    CCP_HIP_CHECK(hipGetDevice(&dev));
    CCP_HIP_CHECK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    const double us = 1e3 / double(khz > 0 ? khz : 100000);
    for (int e = 0; e < 4; ++e) out[e] = double(h[e]) * us;
    out[4] = double(h[4]);
    out[5] = double(df_grid(c, true));
    return CC_OK;
}

int cc_status(cc_ctx *c) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if ((rc = check_dataflow(c))) return rc;
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    return CC_OK;
}

int cc_sweep_rounds(cc_ctx *c, void *x, void *y, const void *g, int32_t first, int32_t count) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(y, "y")) || (rc = need(g, "g")))
        return rc;
    if (first < 0 || count < 0 || first + count > c->nrounds)
        return fail(CC_EINVAL, "round range outside the schedule");
    if (c->prec == CC_F64)
        return sweep_rounds_t<double>(c, (double *)x, (double *)y, (const double *)g, first, count);
    return sweep_rounds_t<float>(c, (float *)x, (float *)y, (const float *)g, first, count);
}

int cc_sweep_metric_prefix(cc_ctx *c, void *x, void *y, const void *g, int32_t nrounds) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(y, "y")) || (rc = need(g, "g")))
        return rc;
    if (nrounds < 0 || nrounds > c->nrounds) return fail(CC_EINVAL, "round count outside the schedule");
    if (!dataflow_b(c->b)) return fail(CC_EINVAL, "the dataflow executor supports b = 8, 16, 24 and 32");
    if (c->prec == CC_F64) return sweep_prefix_t<double>(c, (double *)x, (double *)y, (const double *)g, nrounds);
    return sweep_prefix_t<float>(c, (float *)x, (float *)y, (const float *)g, nrounds);
}

int cc_pair_pass(cc_ctx *c, void *x, void *f, void *yp, const void *g, const uint8_t *d) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(f, "f")) ||
        (rc = need(yp, "y_pair")) || (rc = need(g, "g")) || (rc = need(d, "d")))
        return rc;
    const int64_t np = num_pairs(c->n);
    if (c->prec == CC_F64)
        return launch_pair_pass<double>(np, (double *)x, (double *)f, (double *)yp,
                                        (const double *)g, d, c->stream);
    return launch_pair_pass<float>(np, (float *)x, (float *)f, (float *)yp, (const float *)g, d,
                                   c->stream);
}

int cc_residuals(cc_ctx *c, const void *x, const void *f, const void *y, const void *yp,
                 const double *w, const uint8_t *d, double gamma, int32_t what, cc_resid *out) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(f, "f")) || (rc = need(w, "w")) ||
        (rc = need(d, "d")) || (rc = need(out, "out")))
        return rc;
    if (!(gamma > 0.0)) return fail(CC_EINVAL, "gamma must be > 0");
    if ((what & (CC_RESID_CS | CC_RESID_DUAL)) && (!y || !yp))
        return fail(CC_EINVAL, "y and y_pair are needed for CC_RESID_CS / CC_RESID_DUAL");
    if ((rc = check_dataflow(c))) return rc;
    if (c->prec == CC_F64)
        return residuals_t<double>(c, (const double *)x, (const double *)f, (const double *)y,
                                   (const double *)yp, w, d, gamma, what, out);
    return residuals_t<float>(c, (const float *)x, (const float *)f, (const float *)y,
                              (const float *)yp, w, d, gamma, what, out);
}

int cc_nearness_init(cc_ctx *c, const double *dv, void *x, void *y) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(dv, "d")) || (rc = need(x, "x")) || (rc = need(y, "y")))
        return rc;
    if (c->prec == CC_F64)
        return launch_nearness_init<double>(num_pairs(c->n), c->slots, dv, (double *)x, (double *)y,
                                            c->stream);
    return launch_nearness_init<float>(num_pairs(c->n), c->slots, dv, (float *)x, (float *)y, c->stream);
}

int cc_nearness_residuals(cc_ctx *c, const void *x, const void *y, const double *w, const double *dv,
                          int32_t what, cc_nresid *out) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(x, "x")) || (rc = need(w, "w")) || (rc = need(dv, "d")) ||
        (rc = need(out, "out")))
        return rc;
    if ((what & (CC_RESID_CS | CC_RESID_DUAL)) && !y)
        return fail(CC_EINVAL, "y is needed for CC_RESID_CS / CC_RESID_DUAL");
    if ((rc = check_dataflow(c))) return rc;
    if (c->prec == CC_F64)
        return nearness_residuals_t<double>(c, (const double *)x, (const double *)y, w, dv, what, out);
    return nearness_residuals_t<float>(c, (const float *)x, (const float *)y, w, dv, what, out);
}

int cc_x_from_y(cc_ctx *c, const void *y, const void *yp, const double *w, double gamma,
                void *x, void *f) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(y, "y")) || (rc = need(yp, "y_pair")) ||
        (rc = need(w, "w")) || (rc = need(x, "x_out")) || (rc = need(f, "f_out")))
        return rc;
    if (!(gamma > 0.0)) return fail(CC_EINVAL, "gamma must be > 0");
    if (c->prec == CC_F64)
        return x_from_y_t<double>(c, (const double *)y, (const double *)yp, w, gamma, (double *)x,
                                  (double *)f);
    return x_from_y_t<float>(c, (const float *)y, (const float *)yp, w, gamma, (float *)x,
                             (float *)f);
}

int cc_duals_to_lex(cc_ctx *c, const void *y, void *ylex) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(y, "y_sched")) || (rc = need(ylex, "y_lex"))) return rc;
    if (c->prec == CC_F64)
        return launch_to_lex<double>(c->d_tiles, c->ntiles, c->b, c->n, (const double *)y,
                                     (double *)ylex, c->stream);
    return launch_to_lex<float>(c->d_tiles, c->ntiles, c->b, c->n, (const float *)y,
                                (float *)ylex, c->stream);
}

int cc_slots_to_lex(cc_ctx *c, const int64_t *slots, int64_t count, int64_t *out) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if (count < 0) return fail(CC_EINVAL, "count must be >= 0");
    if (count && ((rc = need(slots, "slots")) || (rc = need(out, "lex_out")))) return rc;
    return launch_slots_to_lex(c->d_tiles, c->ntiles, c->b, c->n, slots, count, out, c->stream);
}

int cc_dataflow_tables(int64_t n, int32_t b, int64_t *ntiles, int64_t *nsteps, int64_t *nblocks,
                       int32_t *tile_pq, uint32_t *need_c, int32_t *jsbase, uint32_t *needs,
                       uint32_t *K) {
    if (n < 3 || b < 1 || b > 32) return fail(CC_EINVAL, "bad n or b");
    std::vector<DTile> tiles;
    std::vector<uint32_t> nd, kk;
    try {
        build_dataflow_tables(n, b, tiles, nd, kk);
    } catch (const std::bad_alloc &) {
        return fail(CC_ENOMEM, "no host memory for the dataflow tables");
    }
    if (ntiles) *ntiles = int64_t(tiles.size());
    if (nsteps) *nsteps = int64_t(nd.size() / 2);
    if (nblocks) *nblocks = int64_t(kk.size());
    for (size_t t = 0; t < tiles.size(); ++t) {
        if (tile_pq) { tile_pq[2 * t] = tiles[t].P; tile_pq[2 * t + 1] = tiles[t].Q; }
        if (need_c) need_c[t] = tiles[t].needC;
        if (jsbase) jsbase[t] = tiles[t].jsbase;
    }
    if (needs) std::memcpy(needs, nd.data(), nd.size() * sizeof(uint32_t));
    if (K) std::memcpy(K, kk.data(), kk.size() * sizeof(uint32_t));
    return CC_OK;
}

int cc_widen(const float *src, double *dst, int64_t count, void *stream) {
    if (count < 0) return fail(CC_EINVAL, "count must be >= 0");
    if (count && (!src || !dst)) return fail(CC_EINVAL, "null pointer");
    return launch_convert<float, double>(count, src, dst, static_cast<hipStream_t>(stream));
}

int cc_narrow(const double *src, float *dst, int64_t count, void *stream) {
    if (count < 0) return fail(CC_EINVAL, "count must be >= 0");
    if (count && (!src || !dst)) return fail(CC_EINVAL, "null pointer");
    return launch_convert<double, float>(count, src, dst, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// ----- learned warm start ----------------------------------------------------
namespace {

int graph_view(cc_ctx *c, const double *w, const uint8_t *d, const float *deg, GraphView &G) {
    if (!c->d_mean_deg && hipMalloc(&c->d_mean_deg, sizeof(float)) != hipSuccess) {
        c->d_mean_deg = nullptr;
        return fail(CC_ENOMEM, "hipMalloc failed");
    }
    int rc = launch_mean_deg(deg, c->n, c->d_mean_deg, c->stream);
    if (rc) return rc;
    G = GraphView{c->d_tiles, c->ntiles, c->b, c->n, w, d, deg, c->d_mean_deg, c->d_chunks, c->nchunks};
    return CC_OK;
}

// Dual objective from the pair state and the metric part of A'y (ax; null
// means zero): D = -b'y - (gamma/2) sum (c + A'y)^2 / w.
template <typename T>
int dual_value(cc_ctx *c, const T *x, const T *f, const T *yp, const double *w, const uint8_t *d,
               const double *ax, double gamma, double *out) {
    int rc = launch_pair_resid<T>(num_pairs(c->n), x, f, yp, w, d, ax, gamma, c->d_ppart, c->stream);
    if (rc) return rc;
    if ((rc = launch_final_reduce(c->d_mpart, 0, c->d_ppart, c->d_out, c->stream))) return rc;
    double h[14];
    CCP_HIP_CHECK(hipMemcpyAsync(h, c->d_out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    if (ax && (rc = check_dataflow(c))) return rc;  // A'y may come from a dataflow launch
    *out = -h[11] - 0.5 * gamma * h[10];
    return CC_OK;
}

// An upper bound on the optimal value of (qp) (= the dual optimum): the
// objective at the best constant point x = c, f = |c - d|, c in [0, 1],
// which satisfies every row (c <= 2c, |x - d| = f).  With W0 and W1 the
// total weight of the positive and the negative pairs,
//   P(c) = c W0 + (1 - c) W1 + (c^2 (W0 + W1) + c^2 W0 + (1 - c)^2 W1) / (2 gamma),
// a convex quadratic, minimised at c = (W1 - gamma (W0 - W1)) / (2 (W0 + W1))
// clipped to [0, 1].
int dual_upper_bound(cc_ctx *c, const double *w, const uint8_t *d, double gamma, double *out) {
    int rc;
    if ((rc = launch_weight_classes(num_pairs(c->n), w, d, c->d_ppart, c->stream))) return rc;
    if ((rc = launch_final_reduce(c->d_mpart, 0, c->d_ppart, c->d_out, c->stream))) return rc;
    double h[14];
    CCP_HIP_CHECK(hipMemcpyAsync(h, c->d_out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    const double W0 = h[5], W1 = h[6];
    double cst = (W1 - gamma * (W0 - W1)) / (2.0 * (W0 + W1));
    cst = std::fmin(1.0, std::fmax(0.0, cst));
    *out = cst * W0 + (1.0 - cst) * W1 +
           (cst * cst * (W0 + W1) + cst * cst * W0 + (1.0 - cst) * (1.0 - cst) * W1) / (2.0 * gamma);
    return CC_OK;
}

// The least share of the gap between the cold start's dual value and the
// bound above that a predicted start must close to be kept.  Hildreth's
// method converges from any y >= 0, but a start that barely raises the
// dual buys no sweeps and costs the inference: measured, the kept starts
// close 14% (n = 2000 planted partition, 40 -> 30 sweeps) and 43% (n = 300
// held-out graphs, 44 -> 20) of that gap, while a network on the n = 4000
// Chung-Lu workload closes 0.3% and then needs 75 sweeps against 70.
constexpr double kGateMinGapShare = 0.05;

// The drawn pairs' terms of the gate: their metric part of A'y at the
// predicted duals (aty, device double[count]) and, if delta is not null,
// their terms of D_warm - D_cold (device double[count]).  The pair kernels
// of the full gate run on the sample in draw order: x = x(y) with zero pair
// duals, one pair pass, from the predicted start and from the cold one.
template <typename T>
int gate_terms_t(cc_ctx *c, const GraphView &G, const float *P, const double *w, const uint8_t *d,
                 double gamma, const T *g, const int64_t *pairs, int64_t count, double *aty,
                 double *delta) {
    int rc;
    if (count <= 0) return CC_OK;
    if ((rc = launch_gate_sample_aty<T>(G, P, pairs, count, aty, c->stream))) return rc;
    if (!delta) return CC_OK;
    const size_t S = size_t(count), al = 256;
    auto up = [&](size_t v) { return (v + al - 1) / al * al; };
    // ws | ds | gs | xw fw xc fc | ypw ypc
    const size_t o_ds = up(S * sizeof(double)), o_gs = o_ds + up(S), o_x = o_gs + up(S * sizeof(T)),
                 o_yp = o_x + 4 * up(S * sizeof(T)), total = o_yp + 2 * up(2 * S * sizeof(T));
    DevTmp t;
    if ((rc = t.alloc(total))) return rc;
    char *base = static_cast<char *>(t.p);
    double *ws = reinterpret_cast<double *>(base);
    uint8_t *ds = reinterpret_cast<uint8_t *>(base + o_ds);
    T *gs = reinterpret_cast<T *>(base + o_gs);
    T *xw = reinterpret_cast<T *>(base + o_x), *fw = reinterpret_cast<T *>(base + o_x + up(S * sizeof(T)));
    T *xc = reinterpret_cast<T *>(base + o_x + 2 * up(S * sizeof(T)));
    T *fc = reinterpret_cast<T *>(base + o_x + 3 * up(S * sizeof(T)));
    T *ypw = reinterpret_cast<T *>(base + o_yp), *ypc = reinterpret_cast<T *>(base + o_yp + up(2 * S * sizeof(T)));
    if ((rc = launch_gate_pairs<T>(num_pairs(c->n), count, pairs, w, d, g, ws, ds, gs, c->stream)) ||
        (rc = launch_init_cold<T>(count, 0, xw, fw, nullptr, ypw, gamma, c->stream)) ||
        (rc = launch_x_from_aty<T>(count, aty, ypw, ws, gamma, xw, fw, c->stream)) ||
        (rc = launch_pair_pass<T>(count, xw, fw, ypw, gs, ds, c->stream)) ||
        (rc = launch_init_cold<T>(count, 0, xc, fc, nullptr, ypc, gamma, c->stream)) ||
        (rc = launch_pair_pass<T>(count, xc, fc, ypc, gs, ds, c->stream)) ||
        (rc = launch_gate_delta<T>(count, aty, ypw, ypc, ws, ds, gamma, delta, c->stream)))
        return rc;
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));  // before the scratch is freed
    return CC_OK;
}

// splitmix64: the pairs the sampled gate draws
uint64_t splitmix64(uint64_t &state) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
constexpr uint64_t kGateSeed = 0x5EED5A3D1E9A7Eull;

// D_warm - D_cold estimated from part of the pairs, with its standard
// error.  The positive pairs (the graph's edges) are few, and the heaviest
// terms sit there: edges at a hub move the most rows.  They are summed
// exactly.  The negative pairs are sampled: gate_sample of them drawn
// uniformly with replacement, their sum estimated as their count times the
// mean term.  On the n = 4000 Chung-Lu workload this stratification cuts
// the standard error 30-fold against a uniform sample of all pairs of the
// same size.  *ran is false when the sample would cost more than 1/8 of the
// full inference, i.e. when 24 (edges + gate_sample) > N_p (each pair
// takes 3 (n - 2) rows of the 3 C(n,3)), when gate_sample is 0, or when the
// host cannot hold the labels and the pair list.
template <typename T>
int gate_estimate_t(cc_ctx *c, const GraphView &G, const float *P, const double *w, const uint8_t *d,
                    double gamma, const T *g, bool *ran, double *est, double *se) {
    *ran = false;
    const int64_t S = c->gate_sample, np = num_pairs(c->n);
    if (S <= 0 || 24.0 * double(S) > double(np)) return CC_OK;
    // host room for the labels and the pair list, else the exact gate alone
    // decides (the estimate only saves time)
    std::vector<uint8_t> hd;
    std::vector<int64_t> pairs;
    std::vector<double> hdl;
    try {
        hd.assign(static_cast<size_t>(np), 0);
    } catch (const std::bad_alloc &) {
        return CC_OK;
    }
    CCP_HIP_CHECK(hipMemcpyAsync(hd.data(), d, size_t(np), hipMemcpyDeviceToHost, c->stream));
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    const int64_t E = int64_t(std::count(hd.begin(), hd.end(), uint8_t(0))), Nn = np - E;
    if (24.0 * double(E + S) > double(np)) return CC_OK;
    try {
        pairs.reserve(static_cast<size_t>(E + S));
        hdl.assign(static_cast<size_t>(E + S), 0.0);
    } catch (const std::bad_alloc &) {
        return CC_OK;
    }
    for (int64_t p = 0; p < np; ++p)
        if (hd[size_t(p)] == 0) pairs.push_back(p);
    // the negative pairs: uniform draws over all pairs, positive ones redrawn
    uint64_t st = kGateSeed;
    for (int64_t k = 0; k < S;) {
        const int64_t p = int64_t(splitmix64(st) % uint64_t(np));
        if (hd[size_t(p)] != 0) {
            pairs.push_back(p);
            ++k;
        }
    }
    const int64_t M = E + S;
    DevTmp t;
    int rc;
    if ((rc = t.alloc(size_t(M) * (sizeof(int64_t) + 2 * sizeof(double))))) return rc;
    int64_t *dp = static_cast<int64_t *>(t.p);
    double *aty = reinterpret_cast<double *>(dp + M), *delta = aty + M;
    CCP_HIP_CHECK(hipMemcpyAsync(dp, pairs.data(), size_t(M) * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    if ((rc = gate_terms_t<T>(c, G, P, w, d, gamma, g, dp, M, aty, delta))) return rc;
    CCP_HIP_CHECK(hipMemcpyAsync(hdl.data(), delta, size_t(M) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    double exact = 0.0, mean = 0.0, var = 0.0;
    for (int64_t e = 0; e < E; ++e) exact += hdl[size_t(e)];
    for (int64_t e = E; e < M; ++e) mean += hdl[size_t(e)];
    mean /= double(S);
    for (int64_t e = E; e < M; ++e) var += (hdl[size_t(e)] - mean) * (hdl[size_t(e)] - mean);
    var = S > 1 ? var / double(S - 1) : 0.0;
    *est = exact + double(Nn) * mean;
    *se = double(Nn) * std::sqrt(var / double(S));
    *ran = true;
    c->gate_drawn = M;
    return CC_OK;
}

template <typename T>
int warm_start_t(cc_ctx *c, const float *P, const float *deg, const double *w, const uint8_t *d,
                 double gamma, T *x, T *f, T *y, T *yp, const T *g, int32_t *accepted,
                 double *dwarm, double *dcold, double *dbound) {
    const int64_t np = num_pairs(c->n);
    GraphView G;
    int rc;
    if ((rc = graph_view(c, w, d, deg, G))) return rc;
    c->gate_drawn = 0;
    c->gate_gain = c->gate_se = 0.0;
    c->gate_rejected = 0;
    // the cold start's value after its first pair pass (metric duals 0), and
    // the bound U: neither depends on the prediction
    double Dw = 0.0, Dc = 0.0, Ub = 0.0;
    {
        DevTmp t0, t1, t2, tz;
        if ((rc = t0.alloc(np * sizeof(T))) || (rc = t1.alloc(np * sizeof(T))) ||
            (rc = t2.alloc(2 * np * sizeof(T))) || (rc = tz.alloc(np * sizeof(double))))
            return rc;
        T *x0 = (T *)t0.p, *f0 = (T *)t1.p, *yp0 = (T *)t2.p;
        CCP_HIP_CHECK(hipMemsetAsync(tz.p, 0, np * sizeof(double), c->stream));
        if ((rc = launch_init_cold<T>(np, c->slots, x0, f0, nullptr, yp0, gamma, c->stream))) return rc;
        if ((rc = launch_pair_pass<T>(np, x0, f0, yp0, g, d, c->stream))) return rc;
        if ((rc = dual_value<T>(c, x0, f0, yp0, w, d, (const double *)tz.p, gamma, &Dc))) return rc;
    }
    if ((rc = dual_upper_bound(c, w, d, gamma, &Ub))) return rc;
    const double need_gain = kGateMinGapShare * (Ub - Dc);
    auto finish = [&](bool ok) {
        if (accepted) *accepted = ok ? 1 : 0;
        if (dwarm) *dwarm = Dw;
        if (dcold) *dcold = Dc;
        if (dbound) *dbound = Ub;
        return CC_OK;
    };
    // An estimate from part of the pairs first (gate_estimate_t): a start
    // whose estimated gain stays below the gate's by four standard errors,
    // and below half of it, is rejected without the full inference.
    bool ran = false;
    double est = 0.0, se = 0.0;
    if ((rc = gate_estimate_t<T>(c, G, P, w, d, gamma, g, &ran, &est, &se))) return rc;
    if (ran) {
        c->gate_gain = est;
        c->gate_se = se;
        if (est + 4.0 * se < need_gain && est < 0.5 * need_gain) {
            c->gate_rejected = 1;
            if ((rc = launch_init_cold<T>(np, c->slots, x, f, y, yp, gamma, c->stream))) return rc;
            CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
            Dw = Dc + est;
            return finish(false);
        }
    }
    // predicted metric duals, pair duals 0, v = v(y), one pair pass
    if (dataflow_b(c->b) && c->iad_grid > 0) {
        // inference fused with A'y: the predictions are summed into the
        // pairs' accumulators as they are written, never read back
        if ((rc = ensure_ax(c))) return rc;
        CCP_HIP_CHECK(hipMemsetAsync(c->d_ax, 0, size_t(np) * sizeof(double), c->stream));
        DataflowArgs a;
        if ((rc = dataflow_args(c, nullptr, a)) || (rc = launch_dataflow_reset(a.ctl, c->stream)) ||
            (rc = launch_infer_aty_dataflow<T>(a, c->iad_grid, G, P, y, c->d_ax, c->stream)))
            return rc;
        c->epoch++;
        if ((rc = launch_init_cold<T>(np, c->slots, x, f, nullptr, yp, gamma, c->stream))) return rc;
        if ((rc = launch_x_from_aty<T>(np, c->d_ax, yp, w, gamma, x, f, c->stream))) return rc;
    } else {
        if ((rc = launch_mlp_infer<T>(G, P, y, c->stream))) return rc;
        if ((rc = launch_init_cold<T>(np, c->slots, x, f, nullptr, yp, gamma, c->stream))) return rc;
        if ((rc = x_from_y_t<T>(c, y, yp, w, gamma, x, f))) return rc;
    }
    if ((rc = launch_pair_pass<T>(np, x, f, yp, g, d, c->stream))) return rc;
    if ((rc = dual_value<T>(c, x, f, yp, w, d, c->d_ax, gamma, &Dw))) return rc;
    const bool ok = std::isfinite(Dw) && Dw - Dc >= need_gain;
    if (!ok && (rc = launch_init_cold<T>(np, c->slots, x, f, y, yp, gamma, c->stream))) return rc;
    return finish(ok);
}

}  // namespace

extern "C" {

int32_t cc_mlp_num_params(void) { return mlp_num_params(); }

int64_t cc_mlp_workspace_bytes(int64_t count) { return int64_t(mlp_workspace_bytes(count)); }

int cc_mlp_init(float *params, uint64_t seed) {
    if (!params) return fail(CC_EINVAL, "null params");
    // He initialisation from a splitmix64 stream (Box-Muller)
    uint64_t st = seed;
    auto next = [&]() {
        st += 0x9E3779B97F4A7C15ull;
        uint64_t z = st;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    auto normal = [&]() {
        const double u1 = next(), u2 = next();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    };
    for (int e = 0; e < 128; ++e) params[e] = float(normal() * std::sqrt(2.0 / 4.0));
    for (int e = 128; e < 160; ++e) params[e] = 0.01f;
    for (int e = 160; e < 1184; ++e) params[e] = float(normal() * std::sqrt(2.0 / 32.0));
    for (int e = 1184; e < 1216; ++e) params[e] = 0.01f;
    for (int e = 1216; e < 1248; ++e) params[e] = float(normal() * std::sqrt(2.0 / 32.0));
    params[1248] = 0.05f;
    return CC_OK;
}

int cc_mlp_forward(const float *params, const float *phi, int64_t count, float *y, void *stream) {
    if (count < 0) return fail(CC_EINVAL, "count must be >= 0");
    if (count && (!params || !phi || !y)) return fail(CC_EINVAL, "null pointer");
    return launch_mlp_forward(params, phi, count, y, static_cast<hipStream_t>(stream));
}

int cc_mlp_train_step(const float *phi, const float *target, int64_t count, float *params,
                      float *adam_m, float *adam_v, int32_t step, float lr, float *grad_out,
                      void *workspace, float *loss_out, void *stream) {
    if (count < 1) return fail(CC_EINVAL, "count must be >= 1");
    if (!phi || !target || !params || !workspace || !loss_out) return fail(CC_EINVAL, "null pointer");
    if (lr > 0.0f && (!adam_m || !adam_v || step < 1)) return fail(CC_EINVAL, "Adam state and step >= 1 needed");
    return launch_mlp_train_explicit(phi, target, count, params, adam_m, adam_v, step, lr, grad_out,
                                     workspace, loss_out, static_cast<hipStream_t>(stream));
}

int cc_mlp_train_graph(cc_ctx *c, const void *ystar, const double *w, const uint8_t *d,
                       const float *deg, int64_t batch, uint64_t seed, float *params, float *adam_m,
                       float *adam_v, int32_t step, float lr, void *workspace, float *loss_out) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(ystar, "y_star")) || (rc = need(w, "w")) ||
        (rc = need(d, "d")) || (rc = need(deg, "deg")) || (rc = need(params, "params")) ||
        (rc = need(workspace, "workspace")) || (rc = need(loss_out, "loss")))
        return rc;
    if (batch < 1) return fail(CC_EINVAL, "batch must be >= 1");
    if (lr > 0.0f && (!adam_m || !adam_v || step < 1)) return fail(CC_EINVAL, "Adam state and step >= 1 needed");
    GraphView G;
    if ((rc = graph_view(c, w, d, deg, G))) return rc;
    if (c->prec == CC_F64)
        return launch_mlp_train_graph<double>(G, (const double *)ystar, c->slots, seed, batch, params,
                                              adam_m, adam_v, step, lr, workspace, loss_out, c->stream);
    return launch_mlp_train_graph<float>(G, (const float *)ystar, c->slots, seed, batch, params,
                                         adam_m, adam_v, step, lr, workspace, loss_out, c->stream);
}

int cc_mlp_slot_features(cc_ctx *c, const double *w, const uint8_t *d, const float *deg,
                         const int64_t *slots, int64_t count, float *phi) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(w, "w")) || (rc = need(d, "d")) || (rc = need(deg, "deg")))
        return rc;
    if (count < 0) return fail(CC_EINVAL, "count must be >= 0");
    if (count && ((rc = need(slots, "slots")) || (rc = need(phi, "phi")))) return rc;
    GraphView G;
    if ((rc = graph_view(c, w, d, deg, G))) return rc;
    return launch_mlp_slot_features(G, slots, count, phi, c->stream);
}

int cc_mlp_infer(cc_ctx *c, const float *params, const float *deg, const double *w,
                 const uint8_t *d, void *y) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(params, "params")) || (rc = need(deg, "deg")) ||
        (rc = need(w, "w")) || (rc = need(d, "d")) || (rc = need(y, "y")))
        return rc;
    GraphView G;
    if ((rc = graph_view(c, w, d, deg, G))) return rc;
    if (c->prec == CC_F64) return launch_mlp_infer<double>(G, params, (double *)y, c->stream);
    return launch_mlp_infer<float>(G, params, (float *)y, c->stream);
}

int cc_warm_start_mlp(cc_ctx *c, const float *params, const float *deg, const double *w,
                      const uint8_t *d, double gamma, void *x, void *f, void *y, void *yp,
                      const void *g, int32_t *accepted, double *dual_warm, double *dual_cold,
                      double *dual_bound) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(params, "params")) || (rc = need(deg, "deg")) ||
        (rc = need(w, "w")) || (rc = need(d, "d")) || (rc = need(x, "x")) || (rc = need(f, "f")) ||
        (rc = need(y, "y")) || (rc = need(yp, "y_pair")) || (rc = need(g, "g")))
        return rc;
    if (!(gamma > 0.0)) return fail(CC_EINVAL, "gamma must be > 0");
    if (c->prec == CC_F64)
        return warm_start_t<double>(c, params, deg, w, d, gamma, (double *)x, (double *)f, (double *)y,
                                    (double *)yp, (const double *)g, accepted, dual_warm, dual_cold,
                                    dual_bound);
    return warm_start_t<float>(c, params, deg, w, d, gamma, (float *)x, (float *)f, (float *)y,
                               (float *)yp, (const float *)g, accepted, dual_warm, dual_cold, dual_bound);
}

int cc_set_gate_sample(cc_ctx *c, int64_t count) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if (count < 0 || count > int64_t(INT32_MAX)) return fail(CC_EINVAL, "count must be in [0, 2^31)");
    c->gate_sample = count;
    return CC_OK;
}

int cc_last_gate_sample(const cc_ctx *c, int64_t *drawn, double *gain, double *std_error,
                        int32_t *rejected) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if (drawn) *drawn = c->gate_drawn;
    if (gain) *gain = c->gate_gain;
    if (std_error) *std_error = c->gate_se;
    if (rejected) *rejected = c->gate_rejected;
    return CC_OK;
}

int cc_warm_gate_terms(cc_ctx *c, const float *params, const float *deg, const double *w,
                       const uint8_t *d, double gamma, const void *g, const int64_t *pairs,
                       int64_t count, double *aty_out, double *delta_out) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = need(params, "params")) || (rc = need(deg, "deg")) ||
        (rc = need(w, "w")) || (rc = need(d, "d")) || (rc = need(g, "g")))
        return rc;
    if (!(gamma > 0.0)) return fail(CC_EINVAL, "gamma must be > 0");
    if (count < 0 || count > int64_t(INT32_MAX)) return fail(CC_EINVAL, "count must be in [0, 2^31)");
    if (count == 0) return CC_OK;
    if ((rc = need(pairs, "pairs")) || (rc = need(aty_out, "aty_out"))) return rc;
    if (c->n < 3) return fail(CC_EINVAL, "no pairs to sample");
    GraphView G;
    if ((rc = graph_view(c, w, d, deg, G))) return rc;
    rc = (c->prec == CC_F64)
             ? gate_terms_t<double>(c, G, params, w, d, gamma, (const double *)g, pairs, count, aty_out,
                                    delta_out)
             : gate_terms_t<float>(c, G, params, w, d, gamma, (const float *)g, pairs, count, aty_out,
                                   delta_out);
    if (rc) return rc;
    CCP_HIP_CHECK(hipStreamSynchronize(c->stream));
    return CC_OK;
}

}  // extern "C"

// ----- one-shot solve ------------------------------------------------------
namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    int alloc(size_t bytes, const char *what) {
        if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) {
            p = nullptr;
            return fail(CC_ENOMEM, std::string("hipMalloc failed for ") + what);
        }
        return CC_OK;
    }
};

struct CtxGuard {
    cc_ctx *c = nullptr;
    ~CtxGuard() { cc_destroy(c); }
};

// Sweeps until both max violations are <= tol (and, with gap_tol > 0, the
// relative duality gap is <= gap_tol) or max_sweeps is reached; returns
// CC_OK or CC_ENOTCONV, *done = sweeps run.  The gap needs A'y, so it is
// evaluated only at checks whose violations already pass.  sparse: sparse
// dual access, with a mask built from y here (nothing else writes y
// meanwhile).  stall > 0: also return CC_OK once the violation is within a
// factor of 100 of tol and `stall` sweeps have passed without a new least
// violation (the FP32 phase of the polish, where rounding may stop the
// progress first; far above tol the violation is not monotone, and there a
// plateau is no stall).
int sweep_to_tol(cc_ctx *c, void *x, void *f, void *y, void *yp, void *g, const uint8_t *d,
                 const double *w, double gamma, double tol, double gap_tol, int max_sweeps,
                 int *done, cc_resid *r, bool sparse, int stall = 0) {
    const int every = c->n <= 1000 ? 1 : 5;
    const int exec = dataflow_b(c->b) ? CC_EXEC_DATAFLOW : CC_EXEC_ROUNDS;
    DevBuf mask;
    if (sparse) {
        int rc;
        if ((rc = mask.alloc(size_t(cc_dual_mask_bytes(c)), "dual mask")) ||
            (rc = cc_dual_mask_build(c, y, mask.p)))
            return rc;
    }
    *done = 0;
    double least = std::numeric_limits<double>::infinity();
    int flat = 0;
    while (*done < max_sweeps) {
        const int k = std::min(every, max_sweeps - *done);
        int rc = sparse ? cc_sweep_sparse(c, x, f, y, yp, g, d, mask.p, k)
                        : cc_sweep(c, x, f, y, yp, g, d, k, exec);
        if (rc) return rc;
        *done += k;
        rc = cc_residuals(c, x, f, nullptr, nullptr, w, d, gamma, CC_RESID_VIOL, r);
        if (rc) return rc;
        const double viol = std::fmax(r->max_viol_metric, r->max_viol_pair);
        if (stall > 0) {
            flat = viol < least ? 0 : flat + k;
            least = std::fmin(least, viol);
            if (flat >= stall && viol <= 100.0 * tol) return CC_OK;
        }
        if (viol <= tol) {
            if (!(gap_tol > 0.0)) return CC_OK;
            rc = cc_residuals(c, x, f, y, yp, w, d, gamma, CC_RESID_VIOL | CC_RESID_DUAL, r);
            if (rc) return rc;
            if (std::fabs(r->gap) <= gap_tol * std::fmax(1.0, std::fabs(r->primal_qp))) return CC_OK;
        }
    }
    return CC_ENOTCONV;
}

}  // namespace

extern "C" int cc_solve_cc_lp(int64_t n, const double *w_host, const uint8_t *d_host,
                              double gamma, double tol, double gap_tol, int32_t max_sweeps,
                              int32_t b, int32_t mode, int32_t warm, const float *mlp_weights_host,
                              const float *deg_host, double *x_out_host,
                              double *y_lex_out_host, cc_info *info) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!w_host || !d_host || !info) return fail(CC_EINVAL, "null w, d or info");
    if (n < 3) return fail(CC_EINVAL, "n must be at least 3");
    if (!(gamma > 0.0) || !std::isfinite(gamma)) return fail(CC_EINVAL, "gamma must be > 0");
    if (!(tol > 0.0)) return fail(CC_EINVAL, "tol must be > 0");
    if (std::isnan(gap_tol)) return fail(CC_EINVAL, "gap_tol must not be NaN");
    if (max_sweeps < 1) return fail(CC_EINVAL, "max_sweeps must be >= 1");
    const bool sparse = (mode & CC_MODE_SPARSE) != 0;
    mode &= ~CC_MODE_SPARSE;
    if (mode != CC_MODE_F64 && mode != CC_MODE_F32 && mode != CC_MODE_F32_POLISH)
        return fail(CC_EINVAL, "unknown mode");
    if (sparse && !dataflow_b(b))
        return fail(CC_EINVAL, "CC_MODE_SPARSE needs b = 8, 16, 24 or 32");
    if (warm != CC_WARM_NONE && warm != CC_WARM_MLP) return fail(CC_EINVAL, "unknown warm start");
    if (warm == CC_WARM_MLP && (!mlp_weights_host || !deg_host))
        return fail(CC_EINVAL, "warm start needs network weights and degrees");
    std::memset(info, 0, sizeof(*info));
    const int64_t np = num_pairs(n);
    for (int64_t p = 0; p < np; ++p)
        if (!(w_host[p] > 0.0) || !std::isfinite(w_host[p]))
            return fail(CC_EINVAL, "every weight must be finite and > 0");

    int rc;
    DevBuf dw, dd;
    if ((rc = dw.alloc(np * sizeof(double), "w")) || (rc = dd.alloc(np, "d"))) return rc;
    CCP_HIP_CHECK(hipMemcpy(dw.p, w_host, np * sizeof(double), hipMemcpyHostToDevice));
    CCP_HIP_CHECK(hipMemcpy(dd.p, d_host, np, hipMemcpyHostToDevice));
    const double *w = static_cast<const double *>(dw.p);
    const uint8_t *d = static_cast<const uint8_t *>(dd.p);

    const bool f32_first = (mode != CC_MODE_F64);
    CtxGuard c32, c64;
    DevBuf x32, f32b, g32, y32, yp32, x64, f64b, g64, y64, yp64;
    cc_resid r{};
    int done = 0, status = CC_OK;

    if (f32_first) {
        if ((rc = cc_create(&c32.c, n, b, CC_F32, nullptr))) return rc;
        const int64_t slots = c32.c->slots;
        if ((rc = x32.alloc(np * 4, "x")) || (rc = f32b.alloc(np * 4, "f")) ||
            (rc = g32.alloc(np * 4, "g")) || (rc = y32.alloc(slots * 4, "y")) ||
            (rc = yp32.alloc(2 * np * 4, "y_pair")))
            return rc;
        if ((rc = cc_prepare(c32.c, w, gamma, g32.p)) ||
            (rc = cc_init_cold(c32.c, x32.p, f32b.p, y32.p, yp32.p, gamma)))
            return rc;
        if (warm == CC_WARM_MLP) {
            DevBuf dP, dDeg;
            if ((rc = dP.alloc(size_t(mlp_num_params()) * sizeof(float), "network")) ||
                (rc = dDeg.alloc(size_t(n) * sizeof(float), "degrees")))
                return rc;
            CCP_HIP_CHECK(hipMemcpy(dP.p, mlp_weights_host, size_t(mlp_num_params()) * sizeof(float),
                                    hipMemcpyHostToDevice));
            CCP_HIP_CHECK(hipMemcpy(dDeg.p, deg_host, size_t(n) * sizeof(float), hipMemcpyHostToDevice));
            int32_t acc = 0;
            rc = cc_warm_start_mlp(c32.c, (const float *)dP.p, (const float *)dDeg.p, w, d, gamma,
                                   x32.p, f32b.p, y32.p, yp32.p, g32.p, &acc, nullptr, nullptr, nullptr);
            if (rc) return rc;
            info->warm_accepted = acc;
            info->warm_sampled = c32.c->gate_rejected;
        }
        // The polish switches to FP64 at max(tol, 1e-5): on the n = 1500
        // Chung-Lu workload an FP32 sweep takes 3.55 ms against 5.94 in FP64
        // and the two phases take 165 sweeps in all wherever the switch lies
        // (1e-4: 105 + 60, 0.77 s; 1e-5: 135 + 30, 0.70 s; 5e-6: 145 + 20,
        // 0.67 s).  1e-5 keeps a factor of 100 over FP32's resolution of x,
        // which lies in [0, 1]; a phase that stops gaining switches earlier.
        const bool polish = (mode == CC_MODE_F32_POLISH);
        const double tol32 = polish ? std::fmax(tol, 1e-5) : tol;
        // the FP32 phase of the polish stops on the violations alone; the
        // FP64 phase applies the gap test
        const double gap32 = polish ? 0.0 : gap_tol;
        status = sweep_to_tol(c32.c, x32.p, f32b.p, y32.p, yp32.p, g32.p, d, w, gamma, tol32, gap32,
                              max_sweeps, &done, &r, sparse, polish ? 20 : 0);
        if (status < 0) return status;
        info->sweeps = info->sweeps_f32 = done;
    }
    if (mode != CC_MODE_F32) {
        if ((rc = cc_create(&c64.c, n, b, CC_F64, nullptr))) return rc;
        const int64_t slots = c64.c->slots;
        if ((rc = x64.alloc(np * 8, "x")) || (rc = f64b.alloc(np * 8, "f")) ||
            (rc = g64.alloc(np * 8, "g")) || (rc = y64.alloc(slots * 8, "y")) ||
            (rc = yp64.alloc(2 * np * 8, "y_pair")))
            return rc;
        if ((rc = cc_prepare(c64.c, w, gamma, g64.p))) return rc;
        if (f32_first) {
            // widen the FP32 duals and rebuild v from them in FP64 (the FP32
            // iterate has drifted from v(y); the duals carry the progress)
            if ((rc = cc_widen((const float *)y32.p, (double *)y64.p, slots, nullptr)) ||
                (rc = cc_widen((const float *)yp32.p, (double *)yp64.p, 2 * np, nullptr)) ||
                (rc = cc_x_from_y(c64.c, y64.p, yp64.p, w, gamma, x64.p, f64b.p)))
                return rc;
        } else {
            if ((rc = cc_init_cold(c64.c, x64.p, f64b.p, y64.p, yp64.p, gamma))) return rc;
            if (warm == CC_WARM_MLP) {
                DevBuf dP, dDeg;
                if ((rc = dP.alloc(size_t(mlp_num_params()) * sizeof(float), "network")) ||
                    (rc = dDeg.alloc(size_t(n) * sizeof(float), "degrees")))
                    return rc;
                CCP_HIP_CHECK(hipMemcpy(dP.p, mlp_weights_host, size_t(mlp_num_params()) * sizeof(float),
                                        hipMemcpyHostToDevice));
                CCP_HIP_CHECK(hipMemcpy(dDeg.p, deg_host, size_t(n) * sizeof(float), hipMemcpyHostToDevice));
                int32_t acc = 0;
                rc = cc_warm_start_mlp(c64.c, (const float *)dP.p, (const float *)dDeg.p, w, d, gamma,
                                       x64.p, f64b.p, y64.p, yp64.p, g64.p, &acc, nullptr, nullptr, nullptr);
                if (rc) return rc;
                info->warm_accepted = acc;
                info->warm_sampled = c64.c->gate_rejected;
            }
        }
        const int left = max_sweeps - info->sweeps;
        if (left > 0) {
            status = sweep_to_tol(c64.c, x64.p, f64b.p, y64.p, yp64.p, g64.p, d, w, gamma, tol,
                                  gap_tol, left, &done, &r, sparse);
            if (status < 0) return status;
            info->sweeps += done;
        } else {
            status = CC_ENOTCONV;
        }
    }
    // final residuals and outputs from the last phase
    cc_ctx *cf = (mode == CC_MODE_F32) ? c32.c : c64.c;
    void *xf = (mode == CC_MODE_F32) ? x32.p : x64.p;
    void *ff = (mode == CC_MODE_F32) ? f32b.p : f64b.p;
    void *yf = (mode == CC_MODE_F32) ? y32.p : y64.p;
    void *ypf = (mode == CC_MODE_F32) ? yp32.p : yp64.p;
    rc = cc_residuals(cf, xf, ff, yf, ypf, w, d, gamma, CC_RESID_ALL, &info->resid);
    if (rc && rc != CC_ENONFINITE) return rc;
    if (rc == CC_ENONFINITE) status = rc;
    if (x_out_host) {
        if (mode == CC_MODE_F32) {
            DevBuf tmp;
            if ((rc = tmp.alloc(np * 8, "x copy"))) return rc;
            if ((rc = cc_widen((const float *)xf, (double *)tmp.p, np, nullptr))) return rc;
            CCP_HIP_CHECK(hipMemcpy(x_out_host, tmp.p, np * 8, hipMemcpyDeviceToHost));
        } else {
            CCP_HIP_CHECK(hipMemcpy(x_out_host, xf, np * 8, hipMemcpyDeviceToHost));
        }
    }
    if (y_lex_out_host) {
        const int64_t nm = cc_num_metric_duals(n);
        DevBuf lex;
        if ((rc = lex.alloc(nm * 8, "y_lex"))) return rc;
        if (mode == CC_MODE_F32) {
            DevBuf lex32;
            if ((rc = lex32.alloc(nm * 4, "y_lex f32"))) return rc;
            if ((rc = cc_duals_to_lex(cf, yf, lex32.p)) ||
                (rc = cc_widen((const float *)lex32.p, (double *)lex.p, nm, nullptr)))
                return rc;
        } else if ((rc = cc_duals_to_lex(cf, yf, lex.p))) {
            return rc;
        }
        CCP_HIP_CHECK(hipMemcpy(y_lex_out_host, lex.p, nm * 8, hipMemcpyDeviceToHost));
    }
    CCP_HIP_CHECK(hipDeviceSynchronize());
    info->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (status == CC_ENOTCONV) set_error("sweep limit reached before the tolerance");
    return status;
}
