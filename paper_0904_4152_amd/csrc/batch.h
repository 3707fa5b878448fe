// Batched execution of many independent mixed-precision multigrid solves
// (persistent stage kernels, per-problem state machine on the device, one
// captured HIP graph per iteration).  Used by mg_solve_batch and the server.
#pragma once

#include <vector>

#include "mg_internal.h"

namespace mg {

// Device view of one level of one problem.
struct BLevel {
    const double* bands64;
    const float* bands32;
    double* x64;
    double* b64;
    float* x32;
    float* b32;
    float* t32;
    int64_t bs;
    int64_t n;
    int N;
    int rh;        // owned rows per fused tile
    int cw;        // owned columns per fused strip
    int bt;        // threads per fused workgroup
    int nstrips;   // fused tiles: nstrips x nchunks
    int nchunks;
    int blk;       // 0: marching tiles; else the block tile shape
};

struct BProb {
    BLevel lv[MG_MAX_LEVEL + 1];
    double* partials;
    dev::CoarseSolver cs;  // coarsest solve
    int L;
    double omega;
    double rel_tol;
    double inner_reduction;
    int inner_max;
    int max_outer;
    int fixed;
    int dmask;  // Dirichlet sides
    int zero_guess;  // x0 = 0, the caller's x not read
};

enum : int {
    BF_INIT = 1,
    BF_OUTER = 2,
    BF_INNER = 8,
    BF_UPDATE = 16,
    BF_DONE = 32
};

struct BState {
    int flags;
    int first;
    int outer;
    int it;
    int cycles;
    int status;
    int n_hist;
    int xnz;  // the initial iterate has a nonzero entry (set by the INIT norm pass)
    double bn, s, dn, r32;
    double hist[MG_HIST];
};

constexpr int ITER_RING = 4;  // iterations whose counts the pinned ring holds

class BatchEngine {
public:
    // capacity problems of levels <= Lmax with common coarse level and
    // smoothing counts.  Allocates device descriptors (not charged: a few MB).
    mg_status init(int device, int capacity, int Lmax, int Lc, int nu_pre, int nu_post);
    ~BatchEngine();

    // Describe slot s (host side); takes effect at the next upload().  b and
    // x (both or neither): the caller's finest right-hand side and iterate,
    // used in place of the hierarchy's (b read; x read unless o.zero_guess,
    // updated in place).
    void set_slot(int s, mg_hierarchy* h, const mg_solve_opts& o, const double* b = nullptr,
                  double* x = nullptr);
    void clear_slot(int s);
    // Mark slot s to start a solve from its hierarchy's finest b64 / x64.
    void start_slot(int s);
    // Upload changed descriptors, work lists and started states; synchronous.
    mg_status upload();
    // The same, stream-ordered (later launches see it; it waits for the work
    // enqueued on setup_stream() so far).
    mg_status upload_async();
    // Asynchronous stepping: launch one iteration; wait for iteration k and
    // read its report (live and certainly-continuing problems, and every
    // slot's flags as of its end, valid until iteration k + ITER_RING is
    // launched).
    mg_status launch_iteration();
    mg_status wait_iteration(int64_t k, int* live, int* sure, const int** flags);
    int64_t launched() const { return launched_; }
    // Device-to-host copies unordered with the iterations, for data of
    // finished problems only.
    mg_status fetch(const void* dev, void* host, size_t bytes);
    mg_status fetch_state(int s, BState* out);
    // Stream for building new problems (assembly); upload_async orders the
    // iterations after it.
    hipStream_t setup_stream() const { return setup_st_; }
    // One iteration over all live slots (graph replay); synchronous.
    mg_status step(int* active_left);
    // Iterations until every slot is done (at most iter_cap), keeping the
    // next needed iteration queued while the host waits; synchronous.
    mg_status run(int64_t iter_cap, int64_t* iterations);
    // Copy the device states to the host mirror; returns it.
    mg_status read_states();
    // After run(): one launch writing x = 0 for the slots whose solution is
    // zero but whose x no update wrote (a zero right-hand side, or a zero
    // guess that stopped before its first update).
    mg_status zero_unwritten();
    // Autotuner: for every level the fused passes run on in the current
    // composition (after upload), time the pre and post passes with each
    // tile height, keep the fastest in the process-wide tile table and
    // report it.  Uses only the FP32 work vectors (scratch); synchronous.
    mg_status tune(int reps, std::vector<mg_tile_choice>* out);
    // Whether tuned workgroup widths apply (default on).  A width change
    // re-captures the iteration graph, so an engine whose composition keeps
    // changing (the server) keeps the width rule; tuned rows always apply.
    void use_tuned_widths(bool on) { tuned_widths_ = on; }
    const BState& state(int s) const { return h_state_[s]; }
    int capacity() const { return cap_; }
    bool live(int s) const { return hp_[s].L > 0; }
    hipStream_t stream() const { return st_; }
    double bytes_per_step() const { return step_bytes_; }

private:
    // with_init: the phase that starts new problems (their ||b||); only the
    // first iteration after an upload that started problems needs it
    hipError_t enqueue_iteration(bool with_init);
    hipError_t launch_fused(int l, bool pre, int mask);
    int problems_at(int l) const;
    void build_lists();
    mg_status ensure_graph();
    mg_status launch();
    mg_status wait(int64_t k, int* live, int* sure);
    int device_ = 0, cap_ = 0, Lmax_ = 0, Lc_ = 1, nu_pre_ = 2, nu_post_ = 2;
    hipStream_t st_ = nullptr;
    BProb* d_probs_ = nullptr;
    BState* d_state_ = nullptr;
    BState* h_state_ = nullptr;  // pinned
    int* d_wl_ = nullptr;
    int* d_iter_ = nullptr;   // iterations run (device counter)
    int* h_ring_ = nullptr;   // pinned: per iteration, live and sure counts
    hipEvent_t ev_[ITER_RING] = {};  // end of the iterations in flight
    int64_t launched_ = 0;    // iterations launched (equals the device counter)
    hipStream_t setup_st_ = nullptr, read_st_ = nullptr;
    hipEvent_t ev_setup_ = nullptr;
    hipEvent_t ev_upload_[2] = {};   // staging area b free again
    int ubuf_ = 0;
    BProb* h_probs_stage_[2] = {};   // pinned staging of descriptors,
    int* h_wl_stage_[2] = {};        // work lists
    BState* h_start_stage_[2] = {};  // and started states
    BState* h_fetch_ = nullptr;      // pinned, one state
    std::vector<BProb> hp_;
    std::vector<int> h_wl_;
    std::vector<char> started_;
    bool probs_dirty_ = true;
    hipGraphExec_t graph_[2] = {};  // iteration graphs without / with the start phase
    bool init_pending_ = false;     // problems started since the last launch
    // Optional launches present in the captured graph: bit l for the fused
    // passes at level l, bit 0 for the residual of problems with no level
    // above the coarse one.  The set only grows (a new bit recaptures).
    uint32_t launch_mask_ = 0;
    double step_bytes_ = 0.0;
    int rh_override_[MG_MAX_LEVEL + 1] = {};  // tile heights under trial (0: none)
    int bt_override_[MG_MAX_LEVEL + 1] = {};  // workgroup widths under trial (0: none)
    int cols_override_[MG_MAX_LEVEL + 1] = {};  // block tile columns under trial (0: march)
    int bt_[MG_MAX_LEVEL + 1] = {};           // workgroup width of each level's fused passes
    int graph_bt_[MG_MAX_LEVEL + 1] = {};     // the widths the captured graph launches
    int blk_[MG_MAX_LEVEL + 1] = {};          // block tile shape of each level's fused passes (0: march)
    int graph_blk_[MG_MAX_LEVEL + 1] = {};    // the shapes the captured graph launches
    bool tuned_widths_ = true;
};



}  // namespace mg
