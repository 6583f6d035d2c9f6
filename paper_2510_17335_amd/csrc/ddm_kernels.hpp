// Kernel launch interface shared by the runtime (ddm_runtime.hip) and the
// kernels (ddm_kernels.hip).  Internal to libddmpm.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddm {

constexpr int kBlock = 256;          // particle kernels: threads per block, and the
                                     // padding unit of every instance's particle range
constexpr int kDetVals = 8;          // partial sums per block in the deterministic mode
constexpr int kNodeVals = 4;         // node record: mv[0..2] (or v), m
constexpr int kPoseVals = 10;        // device pose row of a sub-step
constexpr int kSkillParams = 5;      // skill parameters of the pose Jacobian (depth, angle, push, displace, push angle)
constexpr int kParams = 4 + kSkillParams;   // gradient entries per instance
constexpr int kTile = 4;             // binning tile edge in cells
constexpr int kWin = kTile + 4;      // LDS window edge in nodes: tile + stencil + 1-cell drift each side

// An occupied tile: slots [start, end) of the sorted state, global tile id.
// Tiles and grid node blocks share one index space: tile t holds the cells
// [4t, 4t + 4) per axis and node block t the nodes [4t, 4t + 4).
struct TileRec { uint32_t start, end, tile; };
// queue (may be NULL): two words {next, done} of a persistent launch, zero
// before the launch and again after it (the last workgroup resets them).
struct TileList { const TileRec* list; const uint32_t* count; uint32_t* queue; };

// Window of a tile in the staging buffer: record r holds kWin^D nodes of
// kNodeVals values (node (l0, l1[, l2]) of the window at ((l0 kWin + l1) kWin + l2)),
// covering grid nodes [4t - 1, 4t + 7) per axis.  tslot[t] is the record of
// tile t, or kNoSlot.
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
struct Staging { void* win; const uint32_t* tslot; };

// Active node blocks of a sub-step: every block that can hold mass.  mask[t]
// is nonzero for listed blocks; list[0 .. *count) holds each such block once.
struct ActiveSet { uint32_t* mask; uint32_t* list; uint32_t* count; };

// Per-instance constants on the device (double; kernels cast to their type).
struct InstDev {
  double mu, lam, alpha, kc;         // Lame constants, alpha_f, cohesion shift k_c
  double mp, Vp, dt;                 // particle mass and volume, sub-step
  double dmu_dE, dmu_dnu, dlam_dE, dlam_dnu, dal_dphi, dkc_dphi;   // chain to (E, nu, phi_deg)
  int64_t off, n;                    // first padded particle slot and particle count
  int64_t goff;                      // first grid node of the instance
  double tip0[3];
};

// Device error word.
struct DevErr {
  unsigned int flags;                // 1: NaN/Inf, 2: stencil left the grid, 4: sigma clamped, 8: EMD (ddm_emd.hip),
                                     // 16: a recorded sub-step had more active blocks than the grid record holds
  unsigned int first_inst;
  unsigned long long clamps;
};

// Configuration passed by value to every kernel.
struct KCfg {
  int dim, n, nlog2, bound, shovel, hm_res, region_sign, n_inst, max_steps;
  int pcontact;                      // particle-level collision after G2P (Algorithm 1)
  int64_t nodes;                     // nodes per instance
  int64_t ntot;                      // padded particle slots (SoA stride)
  double dx, inv_dx, gravity, skin, mu_b, half[3];
  double hm_ox, hm_oz, hm_pix, hm_off, region_depth;
  double w_hm, w_mass, m_target, m_ref;
  double w_emd;
  int det;                           // deterministic mode: fixed-order window and reduction sums
};

// Node of an active-set item: item i is node i % 4^D of listed block i / 4^D.
template <int D>
__device__ __forceinline__ void active_node(const KCfg& c, uint32_t gb, int k, int& inst, int idx[3], int64_t& node) {
  // grids are powers of two: blocks per axis 2^tb, blocks per instance 2^(D tb)
  const int tb = c.nlog2 - 2, pb = D * tb;
  const uint32_t mb = (1u << tb) - 1u;
  inst = (int)(gb >> pb);
  const uint32_t t = gb & ((1u << pb) - 1u);
  int bc[3] = {0, 0, 0};
  if (D == 3) { bc[0] = (int)(t >> (2 * tb)); bc[1] = (int)((t >> tb) & mb); bc[2] = (int)(t & mb); }
  else { bc[0] = (int)(t >> tb); bc[1] = (int)(t & mb); }
  if (D == 3) { idx[0] = bc[0] * kTile + (k >> 4); idx[1] = bc[1] * kTile + ((k >> 2) & 3); idx[2] = bc[2] * kTile + (k & 3); }
  else { idx[0] = bc[0] * kTile + (k >> 2); idx[1] = bc[1] * kTile + (k & 3); idx[2] = 0; }
  node = D == 3 ? ((int64_t)idx[0] << (2 * c.nlog2)) + ((int64_t)idx[1] << c.nlog2) + idx[2]
                : ((int64_t)idx[0] << c.nlog2) + idx[1];
}

// Pointers of one launch.
struct Bufs {
  const InstDev* inst;
  const int* blk_inst;               // instance of every particle block
  const void* poses;                 // [n_inst][max_steps][kPoseVals]: tip xyz, psi, vel xyz, omega, sin psi, cos psi
  DevErr* err;
  // deterministic mode: 8 partial sums per particle block or per grid block,
  // all zero between uses (each reduction's finish clears what it read); NULL
  // otherwise (reductions add with atomics)
  double* dpart = nullptr;
};

// Deterministic reductions: adds to dst[i * stride + k] (k < nvals) the
// partials of instance i in dpart, summed in a fixed order, and zeroes them.
// grid_blocks: the partials are indexed by global node block (instance i owns
// blocks [i per, (i + 1) per)); otherwise by particle block.
void launch_det_finish(const KCfg& c, const Bufs& b, bool grid_blocks, int nvals, double* dst, int64_t stride,
                       hipStream_t s);

// Forward sub-step pieces.  state_* are SoA particle states (stride ntot).
void launch_fill_zero(void* p, int64_t count, int elem_bytes, hipStream_t s);
// Per-instance diagnostics of the state and of the last grid (grid_pre may be
// NULL: no grid), DDM_N_DIAG doubles per instance (ddm_diag.hip).
void launch_diagnostics(int prec, const KCfg& c, const Bufs& b, int nblk, const void* state, const void* grid_pre,
                        const ActiveSet& act, double* out, hipStream_t s);
void launch_eval_math(int fn, const float* x, float* y, int64_t n, hipStream_t s);
void launch_fill_u32(void* p, int64_t words, uint32_t value, hipStream_t s);
// Particle state from positions x0[n][D] (instances concatenated): v = 0, C = 0,
// G = 0 and ids; positions_only writes the position rows and ids alone.
void launch_init_state(int prec, const KCfg& c, const Bufs& b, int nblk, const void* x0, void* state,
                       uint32_t* pid, hipStream_t s, bool positions_only = false);
// Up to kBlobWords * 4 bytes from host memory to device memory, carried in the
// arguments of a one-block kernel (no host buffer has to outlive the call).
constexpr int kBlobWords = 128;
void launch_put_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);
// P2G writes every occupied tile's window to the staging buffer; particles
// that left their window add to the dense outlier grid gout (kept zero
// otherwise) and add their node blocks to the active set.
// tau_out (may be NULL): the Kirchhoff stress of every particle, symmetric
// rows (00, 01, 02, 11, 12, 22; 2D: 00, 01, 11) of stride ntot, for the reverse pass.
void launch_p2g(int prec, const KCfg& c, const Bufs& b, const TileList& tl, int nwg, const void* st_in, void* st_out,
                const Staging& stg, void* gout, const ActiveSet& act, void* tau_out, hipStream_t s);
// Grid update over the active blocks: sums the staged windows and the outlier
// grid (zeroing what it read) into grid_pre (m, mv), writes grid_post (v, m).
// pre_cap < 0: grid_pre is the dense grid; pre_cap >= 0: grid_pre is a record
// of pre_cap node entries in the order of the active list (more flag bit 4).
// list_out / count_out (may be NULL) receive a copy of the active list.
// The post-update grid of sub-step `step` rebuilt from the record of its
// pre-update grid (pre_cap entries) over the listed active blocks (list,
// count: as the grid update wrote them); pre_dense (may be NULL) also
// receives the pre-update values at their grid positions.
void launch_grid_post_from_pre(int prec, const KCfg& c, const Bufs& b, int step, const uint32_t* list,
                               const uint32_t* count, const void* pre, int64_t pre_cap, void* post, void* pre_dense,
                               hipStream_t s);
void launch_grid_update(int prec, const KCfg& c, const Bufs& b, int step, const Staging& stg, void* gout,
                        const ActiveSet& act, void* grid_pre, int64_t pre_cap, void* grid_post, uint32_t* list_out,
                        uint32_t* count_out, hipStream_t s);
// Active set of a fresh binning: the blocks of the occupied tiles and of their
// neighbours (a tile's window reaches one block beyond it on each side).
void launch_active_set(const KCfg& c, const TileList& tl, const ActiveSet& act, hipStream_t s);
// G2P of sub-step `step`, with the particle-level collision when c.pcontact.
void launch_g2p(int prec, const KCfg& c, const Bufs& b, int nblk, int step, const void* st_in, void* st_out,
                const void* grid_post, hipStream_t s);
void launch_export_state(const KCfg& c, const Bufs& b, int nblk, int rows, int elem_bytes, const void* in, void* out,
                         const uint32_t* pid, hipStream_t s);
void launch_reset_pid(const Bufs& b, int nblk, uint32_t* pid, hipStream_t s);
void launch_grid_export(int prec, const KCfg& c, const void* grid_pre, const void* grid_post, const uint32_t* mask,
                        void* out, hipStream_t s);

// Loss (height map + scoop mass) and its seed adjoint.
struct LossBufs {
  unsigned long long* hm_bits;       // [n_inst][npix] max height as ordered bits
  unsigned int* owner;               // [n_inst][npix] lowest particle id at the max
  const double* target;              // [n_inst][npix]
  double* hm_val;                    // [n_inst][npix]
  double* dldh;                      // [n_inst][npix]
  double* region;                    // [n_inst] scoop mass
  double* dldm;                      // [n_inst]
  double* loss;                      // [n_inst]
};
void launch_loss(int prec, const KCfg& c, const Bufs& b, int nblk, const void* state, const uint32_t* pid,
                 int final_step, const LossBufs& L, hipStream_t s);
void launch_loss_seed(int prec, const KCfg& c, const Bufs& b, int nblk, const void* state, const uint32_t* pid,
                      int final_step, const LossBufs& L, void* adj, double* pacc, hipStream_t s);

// Adjoint sub-step pieces (reverse order: g2p_adj, grid_adj, p2g_adj).
// stg (may be NULL): the deterministic mode's staging records, one per listed
// tile, which receive each tile's window instead of atomics into gvb; then
// launch_adj_windows adds them to gvb (tslot: the record of each tile of the
// sub-step's list, as launch_tile_slots builds it).
void launch_g2p_adj(int prec, const KCfg& c, const Bufs& b, const TileList& tl, int nwg, const void* st,
                    const void* grid_post, const void* adj_next, void* adj_cur, void* gvb, void* stg, hipStream_t s);
void launch_adj_windows(int prec, const KCfg& c, const Bufs& b, const uint32_t* list, const uint32_t* count,
                        const void* stg, const uint32_t* tslot, void* gvb, hipStream_t s);
// Adjoint of the particle-level collision of sub-step `step` (run before the
// G2P adjoint when c.pcontact): rewrites the x and v rows of adj_next so that
// the G2P adjoint sees the adjoint of the velocity before the collision, adds
// the collision's position adjoint to x, and adds its pose adjoints to pose_bar.
void launch_pcontact_adj(int prec, const KCfg& c, const Bufs& b, int nblk, int step, const void* st,
                         const void* grid_post, void* adj_next, double* pose_bar, hipStream_t s);
// Over the active blocks (list, count) of the sub-step, with the record of
// its pre-update grid (pre_cap entries in list order); zeroes gvb where it
// read it.
void launch_grid_adj(int prec, const KCfg& c, const Bufs& b, int step, const uint32_t* list, const uint32_t* count,
                     const void* grid_pre, int64_t pre_cap, void* gvb, void* gb, double* pose_bar, hipStream_t s);
// stress_form: the density adjoint of the sub-step as -sum_p (S_p : A bar_p) / rho,
// S_p the stress part of A_p (valid while the grid adjoints are untreated,
// where m bar = -v bar . (mv/m) / m holds); otherwise from the grid mass adjoint.
void launch_p2g_adj(int prec, const KCfg& c, const Bufs& b, int nblk, const void* st, const void* tau, const void* gb,
                    bool stress_form, const void* adj_next, void* adj_cur, double* pacc, hipStream_t s);
void launch_grad_final(const KCfg& c, const InstDev* inst, const double* pacc, const double* pose_bar,
                       const double* pose_jac, int n_steps, const double* dloss, double* grad, hipStream_t s);

// Binning (ddm_sort.hip).
// Cell keys of the particles in slot order, or of the particles order[j]
// (order may be NULL); vals receive the particle slots.
void launch_keys(int prec, const KCfg& c, const Bufs& b, int nblk, const void* state, uint32_t* keys, uint32_t* vals,
                 hipStream_t s, const uint32_t* order = nullptr);
void launch_pid_keys(const uint32_t* pid, uint32_t* keys, uint32_t* vals, int64_t ntot, hipStream_t s);
int sort_passes(uint32_t max_key);
int64_t sort_hist_words(int64_t n);
int64_t sort_sum_words(int64_t n);
int radix_sort(uint32_t* keys[2], uint32_t* vals[2], int64_t n, uint32_t max_key, uint32_t* hist, uint32_t* sums,
                hipStream_t s);
void launch_gather(int elem_bytes, const void* in, void* out, const uint32_t* perm, int rows, int64_t ntot,
                   const uint32_t* pid_in, uint32_t* pid_out, hipStream_t s);
void launch_unpermute(int elem_bytes, const void* in, void* out, const uint32_t* perm, int rows, int64_t ntot,
                      hipStream_t s);
// tslot of a recorded tile list: tslot[list[r].tile] = r, kNoSlot elsewhere.
void launch_tile_slots(const KCfg& c, const TileList& tl, int64_t max_records, uint32_t* tslot, hipStream_t s);
// One record per occupied tile, largest particle count first (bucket: 2
// kTileBuckets words of scratch), and tslot (record of each tile, or kNoSlot).
constexpr int kTileBuckets = 16;
void launch_tile_list(const KCfg& c, const uint32_t* sorted_keys, uint32_t* tstart, uint32_t* tend, TileRec* list,
                      uint32_t* count, uint32_t* tslot, uint32_t* bucket, hipStream_t s);

// Earth mover's distance of the surface observation to a target point cloud
// (ddm_emd.hip); arrays are [n_inst][hm_res^2] (points [..][3]).
struct EmdBufs {
  unsigned long long* top;        // highest position key per pixel
  unsigned long long* own;        // (particle id << 32 | slot) of the pixel's owner, ~0 if none
  double* target;                 // target points, m per instance
  double* obs;                    // observed points, pixel order
  int* obs_slot;                  // owner slot of each observed point (relative to the instance)
  int* n_obs;                     // [n_inst]
  int* assign;                    // target of each observed point
  double* emd;                    // [n_inst]
};
constexpr int kEmdMaxPoints = 4096;   // observed and target points per instance (hm_res <= 64)
// loss[inst] += w_emd * EMD of the state (the targets hold m points per instance).
void launch_emd(int prec, const KCfg& c, const Bufs& b, int nblk, const void* state, const uint32_t* pid,
                const EmdBufs& E, int m, double w_emd, double* loss, hipStream_t s);
// adjoint x rows += w_emd * d EMD / d x (after the loss seed).
void launch_emd_seed(int prec, const KCfg& c, const Bufs& b, const EmdBufs& E, double w_emd, void* adj,
                     hipStream_t s);

// Gradient treatments of the reverse pass (ddm_treat.hip).  Variables (one
// vector per instance each): 0 particle x, 1 particle v, 2 particle F, 3 grid
// velocity after the grid update, 4 grid momentum, 5 grid mass.  acc holds
// treat_acc_words(n_inst) 64-bit words, [n_inst][variable][phase][3], zeroed
// before each reduction; phase 0 is reduced before a treatment, phase 1 after it.
constexpr int kTreatVars = 6;
constexpr int kTreatNone = 0, kTreatClip = 1, kTreatScale = 2, kTreatNorm = 3;
struct Treat { int mode; double clip, oom, delta; };
size_t treat_acc_words(int n_inst);
// The treatment of the particle adjoints (x, v, F) and of one grid buffer
// (variable var, and var + 1 for value 3 of a node when with_mass), with the
// statistics before and after it into acc when record is set.
void launch_treat_particles(int prec, const KCfg& c, const Bufs& b, int nblk, void* adj, const Treat& t, bool record,
                            unsigned long long* acc, hipStream_t s);
void launch_treat_grid(int prec, const KCfg& c, const Bufs& b, const uint32_t* list, const uint32_t* count, void* g,
                       int var, bool with_mass, const Treat& t, bool record, unsigned long long* acc, hipStream_t s);
// out[n_inst][kTreatVars][6]: max, min, 2-norm before the treatment and after it.
void launch_treat_record(int n_inst, const unsigned long long* acc, bool post, double* out, hipStream_t s);

}  // namespace ddm
