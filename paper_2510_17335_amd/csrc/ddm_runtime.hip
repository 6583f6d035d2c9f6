// Host runtime of libddmpm.so: validation, workspace layout, the digging
// skill's pose tables, the rollout with checkpoints and the reverse pass, and
// the C interface declared in include/ddmpm.h.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ddmpm.h"
#include "ddm_kernels.hpp"

// A roctx range over one phase of the library (host-side marker: a
// `rocprofv3 --marker-trace` run shows rollouts, replays and reverse passes
// as named spans; without a profiler the calls return at once).
struct Phase {
  bool on;
  explicit Phase(const char* name, bool active = true) : on(active) { if (on) roctxRangePushA(name); }
  ~Phase() { if (on) roctxRangePop(); }
  Phase(const Phase&) = delete;
  Phase& operator=(const Phase&) = delete;
};

namespace {

thread_local std::string g_last_error;

ddm_status fail(ddm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

ddm_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return DDM_OK;
  return fail(DDM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define DDM_HIP(call)                                   \
  do {                                                  \
    ddm_status _s = hip_check((call), #call);           \
    if (_s != DDM_OK) return _s;                        \
  } while (0)

constexpr double kPi = 3.14159265358979323846;

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

int64_t pad_up(int64_t n, int64_t m) { return (n + m - 1) / m * m; }

// Device workspace carved into 256-byte aligned pieces.
struct Layout {
  size_t inst = 0, blk_inst = 0, poses = 0, pose_jac = 0, err = 0, pid = 0, pid_tmp = 0;
  size_t cur = 0, grid_pre = 0, grid_post = 0, scratch = 0;
  size_t ckpt = 0, seg_state = 0, seg_grid = 0, seg_tau = 0, seg_perm = 0, seg_tiles = 0, seg_tcount = 0;
  size_t tau_bytes = 0;
  size_t adj0 = 0, adj1 = 0, gvb = 0, gb = 0, pacc = 0, pose_bar = 0;
  size_t hm_bits = 0, owner = 0, target = 0, hm_val = 0, dldh = 0, region = 0, dldm = 0, loss = 0;
  size_t keys0 = 0, keys1 = 0, vals0 = 0, vals1 = 0, hist = 0, sums = 0, tstart = 0, tend = 0, tiles = 0, tcount = 0;
  size_t tslot = 0, tbucket = 0, staging = 0, gout = 0, amask = 0, alist = 0, acount = 0, seg_alist = 0, seg_acount = 0;
  size_t treat_acc = 0, tqueue = 0, dpart = 0, ckpt_pid = 0, rpid0 = 0, rpid1 = 0;
  size_t emd_top = 0, emd_own = 0, emd_target = 0, emd_obs = 0, emd_slot = 0, emd_nobs = 0, emd_assign = 0,
         emd_val = 0;
  size_t total = 0;
  size_t state_bytes = 0, grid_bytes = 0;
  int64_t rec_items = 0;              // node entries of one sub-step's pre-update grid record
  size_t rec_bytes = 0;               // bytes of that record
  int64_t ntot = 0, nblk = 0, total_tiles = 0, max_chunks = 0;
  size_t win_bytes = 0;               // one staged window
  int n_ckpt = 0, K = 1, rows = 0, esz = 4, nwg = 1;
  int M = 1;                          // sets of segment buffers
  size_t seg_set = 0;                 // bytes of one set (sets follow each other)
  uint32_t max_key = 0;
};

struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    off = (off + 255) / 256 * 256;
    const size_t o = off;
    off += bytes;
    return o;
  }
};

Layout make_layout(const ddm_config& c, int n_inst, const ddm_instance* in) {
  Layout L;
  const int D = c.dim;
  const int b = c.precision == DDM_F64 ? 8 : 4;
  int64_t ntot = 0;
  for (int i = 0; i < n_inst; ++i) ntot += pad_up(in[i].n_particles, ddm::kBlock);
  L.ntot = ntot;
  L.nblk = ntot / ddm::kBlock;
  int64_t nodes = 1;
  for (int a = 0; a < D; ++a) nodes *= c.n_grid;
  const int S = 2 * D + 2 * D * D;
  L.rows = S;
  L.esz = b;
  L.state_bytes = (size_t)S * ntot * b;
  const int64_t tiles_per_inst = nodes / (D == 3 ? ddm::kTile * ddm::kTile * ddm::kTile : ddm::kTile * ddm::kTile);
  L.total_tiles = tiles_per_inst * n_inst;
  L.max_key = (uint32_t)((uint64_t)n_inst * (uint64_t)(nodes + 1) - 1);
  // One record per occupied tile.  Workgroups of the tile kernels: about one
  // per expected occupied tile, grid-stride beyond that.
  L.max_chunks = L.total_tiles;
  L.nwg = (int)std::max<int64_t>(1, std::min<int64_t>(L.total_tiles, L.nblk + 1024));
  L.win_bytes = (size_t)ddm::kNodeVals * (D == 3 ? ddm::kWin * ddm::kWin * ddm::kWin : ddm::kWin * ddm::kWin) * b;
  L.grid_bytes = (size_t)n_inst * nodes * ddm::kNodeVals * b;
  L.K = std::max(1, (int)c.checkpoint_every);
  L.n_ckpt = (c.max_steps + L.K - 1) / L.K + 1;
  const int npix = D == 3 ? c.hm_res * c.hm_res : c.hm_res;
  Carver cv;
  L.inst = cv.take(sizeof(ddm::InstDev) * n_inst);
  L.blk_inst = cv.take(sizeof(int) * L.nblk);
  L.poses = cv.take((size_t)n_inst * c.max_steps * ddm::kPoseVals * b);
  L.pose_jac = cv.take((size_t)n_inst * c.max_steps * 8 * ddm::kSkillParams * sizeof(double));
  L.err = cv.take(sizeof(ddm::DevErr));
  L.tqueue = cv.take(2 * sizeof(uint32_t));
  L.pid = cv.take(sizeof(uint32_t) * ntot);
  L.pid_tmp = cv.take(sizeof(uint32_t) * ntot);
  L.cur = cv.take(L.state_bytes);
  L.scratch = cv.take(L.state_bytes);
  L.grid_pre = cv.take(L.grid_bytes);
  L.grid_post = cv.take(L.grid_bytes);
  L.ckpt = cv.take(L.state_bytes * L.n_ckpt);
  // Segment buffers: the reverse pass's record of one checkpoint segment
  // (per sub-step the state, the pre-update grid, the stress, the binning
  // permutation, the tile list and the active blocks; the post-update grid is
  // rebuilt from the pre-update one when needed), M sets back to back.
  L.tau_bytes = (size_t)(D * (D + 1) / 2) * ntot * b;
  L.M = std::max(1, std::min<int>(c.record_segments, (c.max_steps + L.K - 1) / L.K));
  const size_t seg0 = cv.take(0);
  L.seg_state = cv.take(L.state_bytes * (L.K + 1));
  {
    const int64_t npb = D == 3 ? ddm::kTile * ddm::kTile * ddm::kTile : ddm::kTile * ddm::kTile;
    const int64_t blocks = c.grid_record_blocks > 0 ? std::min<int64_t>(c.grid_record_blocks, L.total_tiles)
                                                     : L.total_tiles;
    L.rec_items = blocks * npb;
    L.rec_bytes = (size_t)L.rec_items * ddm::kNodeVals * b;
  }
  L.seg_grid = cv.take(L.rec_bytes * L.K);
  L.seg_tau = cv.take(L.tau_bytes * L.K);
  L.seg_perm = cv.take(sizeof(uint32_t) * ntot * L.K);
  L.seg_tiles = cv.take(sizeof(ddm::TileRec) * L.max_chunks * L.K);
  L.seg_tcount = cv.take(sizeof(uint32_t) * L.K);
  L.seg_alist = cv.take(sizeof(uint32_t) * L.total_tiles * L.K);
  L.seg_acount = cv.take(sizeof(uint32_t) * L.K);
  L.seg_set = cv.take(0) - seg0;
  cv.take(L.seg_set * (L.M - 1));
  L.adj0 = cv.take(L.state_bytes);
  L.adj1 = cv.take(L.state_bytes);
  L.gvb = cv.take(L.grid_bytes);
  L.gb = cv.take(L.grid_bytes);
  L.pacc = cv.take(sizeof(double) * 8 * n_inst);
  L.treat_acc = cv.take(sizeof(unsigned long long) * ddm::treat_acc_words(n_inst));
  L.pose_bar = cv.take(sizeof(double) * 8 * (size_t)n_inst * c.max_steps);
  L.hm_bits = cv.take(sizeof(unsigned long long) * (size_t)n_inst * npix);
  L.owner = cv.take(sizeof(unsigned int) * (size_t)n_inst * npix);
  L.target = cv.take(sizeof(double) * (size_t)n_inst * npix);
  L.hm_val = cv.take(sizeof(double) * (size_t)n_inst * npix);
  L.dldh = cv.take(sizeof(double) * (size_t)n_inst * npix);
  L.region = cv.take(sizeof(double) * n_inst);
  L.dldm = cv.take(sizeof(double) * n_inst);
  L.loss = cv.take(sizeof(double) * n_inst);
  L.keys0 = cv.take(sizeof(uint32_t) * ntot);
  L.keys1 = cv.take(sizeof(uint32_t) * ntot);
  L.vals0 = cv.take(sizeof(uint32_t) * ntot);
  L.vals1 = cv.take(sizeof(uint32_t) * ntot);
  L.hist = cv.take(sizeof(uint32_t) * ddm::sort_hist_words(ntot));
  L.sums = cv.take(sizeof(uint32_t) * ddm::sort_sum_words(ddm::sort_hist_words(ntot)));
  L.tstart = cv.take(sizeof(uint32_t) * L.total_tiles);
  L.tend = cv.take(sizeof(uint32_t) * L.total_tiles);
  L.tiles = cv.take(sizeof(ddm::TileRec) * L.max_chunks);
  L.tcount = cv.take(sizeof(uint32_t));
  L.tslot = cv.take(sizeof(uint32_t) * L.total_tiles);
  L.tbucket = cv.take(sizeof(uint32_t) * 2 * ddm::kTileBuckets);
  L.staging = cv.take(L.win_bytes * L.total_tiles);
  L.gout = cv.take(L.grid_bytes);
  L.amask = cv.take(sizeof(uint32_t) * L.total_tiles);
  L.alist = cv.take(sizeof(uint32_t) * L.total_tiles);
  L.acount = cv.take(sizeof(uint32_t));
  // deterministic mode: partial sums per particle block or grid block
  if (c.deterministic) {
    L.dpart = cv.take(sizeof(double) * ddm::kDetVals * (size_t)std::max(L.nblk, L.total_tiles));
    // the particle ids at every checkpoint and a pair for the replays: a cell's
    // particles are ordered by id at every binning
    L.ckpt_pid = cv.take(sizeof(uint32_t) * (size_t)ntot * L.n_ckpt);
    L.rpid0 = cv.take(sizeof(uint32_t) * (size_t)ntot);
    L.rpid1 = cv.take(sizeof(uint32_t) * (size_t)ntot);
  }
  if (D == 3 && c.w_emd != 0.0) {
    const size_t np = (size_t)n_inst * c.hm_res * c.hm_res;
    L.emd_top = cv.take(8 * np);
    L.emd_own = cv.take(8 * np);
    L.emd_target = cv.take(24 * np);
    L.emd_obs = cv.take(24 * np);
    L.emd_slot = cv.take(4 * np);
    L.emd_nobs = cv.take(4 * (size_t)n_inst);
    L.emd_assign = cv.take(4 * np);
    L.emd_val = cv.take(8 * (size_t)n_inst);
  }
  L.total = cv.take(0);
  return L;
}

// ---------------------------------------------------------------------------
// Digging skill (Sec. III-B): phase lengths T_i = round(T^float_i) (half away
// from zero, no derivative), per-action displacements of the four phases, and
// the per-sub-step blade pose: the action is spread evenly over the n_sub
// sub-steps and applied before the grid collision (the agent move of Algorithm 1).  With
// skill_unrounded the steps of phases 1 and 4 divide by T^float_1, T^float_4
// instead (the alternative mapping; its derivative is carried), where max()
// keeps its first argument on ties.  Build frame: paper (x, y, z) -> (x, z,
// y), rotation about the paper's x axis -> psi.  Jacobian columns:
// d/d(depth, angle_deg, push, displace, push_angle_deg).
// ---------------------------------------------------------------------------
constexpr int kSkill = ddm::kSkillParams;
struct Action { double d[6]; double J[6][kSkill]; };   // paper frame [dx, dy, dz, drx, dry, drz]

std::vector<Action> skill_actions(const ddm_config& c, const ddm_instance& in) {
  const double dta = c.n_sub * in.dt;
  const double rad = kPi / 180.0;
  const double phi1 = in.angle_deg * rad, d1 = in.displace, d2 = in.depth, d3 = in.push, d4 = c.d_lift;
  const double phi3 = in.push_angle_deg * rad;
  const bool unr = c.skill_unrounded != 0;
  // T^float with their derivatives in (d1, phi1_deg): |d1| / (v_l dta), |phi1| / (v_w dta)
  const double Tf_d1 = std::fabs(d1) / (c.v_lin * dta), Tf_phi1 = std::fabs(phi1) / (c.v_ang * dta);
  const double dTd1 = (d1 >= 0 ? 1.0 : -1.0) / (c.v_lin * dta);            // d Tf_d1 / d d1
  const double dTphi = (phi1 >= 0 ? 1.0 : -1.0) * rad / (c.v_ang * dta);   // d Tf_phi1 / d angle_deg
  const bool t1_by_d1 = Tf_d1 >= Tf_phi1;
  const double Tf1 = t1_by_d1 ? Tf_d1 : Tf_phi1;
  const double Tf_lift = d4 / (c.v_lin * dta);
  const bool t4_by_phi = Tf_phi1 >= Tf_lift;
  const double Tf4 = t4_by_phi ? Tf_phi1 : Tf_lift;
  const long T1 = std::lround(Tf1);
  const long T2 = std::lround(d2 / (c.v_lin * dta));
  const long T3 = std::lround(std::fabs(d3 / (c.v_lin * dta)));
  const long T4 = std::lround(Tf4);
  const double phi2 = phi1 + kPi / 2.0;
  std::vector<Action> out;
  auto blank = [] { Action a; std::memset(&a, 0, sizeof(a)); return a; };
  enum { DEPTH = 0, ANGLE = 1, PUSH = 2, DISP = 3, PANG = 4 };
  // phase 1: (d1, phi1) / div1, div1 = T1 or Tf1
  const double div1 = unr ? Tf1 : (double)T1;
  double ddiv1[kSkill] = {0, 0, 0, 0, 0};
  if (unr) { if (t1_by_d1) ddiv1[DISP] = dTd1; else ddiv1[ANGLE] = dTphi; }
  for (long t = 0; t < T1; ++t) {
    Action a = blank();
    a.d[0] = d1 / div1;
    a.d[3] = phi1 / div1;
    for (int j = 0; j < kSkill; ++j) {
      a.J[0][j] = -d1 * ddiv1[j] / (div1 * div1);
      a.J[3][j] = -phi1 * ddiv1[j] / (div1 * div1);
    }
    a.J[0][DISP] += 1.0 / div1;
    a.J[3][ANGLE] += rad / div1;
    out.push_back(a);
  }
  for (long t = 0; t < T2; ++t) {
    Action a = blank();
    a.d[0] = d2 * std::cos(phi2) / T2;
    a.d[2] = -(d2 * std::sin(phi2)) / T2;
    a.J[0][DEPTH] = std::cos(phi2) / T2;
    a.J[0][ANGLE] = -d2 * std::sin(phi2) * rad / T2;
    a.J[2][DEPTH] = -std::sin(phi2) / T2;
    a.J[2][ANGLE] = -d2 * std::cos(phi2) * rad / T2;
    out.push_back(a);
  }
  for (long t = 0; t < T3; ++t) {
    Action a = blank();
    a.d[0] = d3 * std::cos(phi3) / T3;
    a.d[2] = d3 * std::sin(phi3) / T3;
    a.J[0][PUSH] = std::cos(phi3) / T3;
    a.J[2][PUSH] = std::sin(phi3) / T3;
    a.J[0][PANG] = -d3 * std::sin(phi3) * rad / T3;
    a.J[2][PANG] = d3 * std::cos(phi3) * rad / T3;
    out.push_back(a);
  }
  // phase 4: (-phi1, d4) / div4, div4 = T4 or Tf4
  const double div4 = unr ? Tf4 : (double)T4;
  const double ddiv4_angle = (unr && t4_by_phi) ? dTphi : 0.0;
  for (long t = 0; t < T4; ++t) {
    Action a = blank();
    a.d[3] = -phi1 / div4;
    a.d[2] = d4 / div4;
    a.J[3][ANGLE] = -rad / div4 + phi1 * ddiv4_angle / (div4 * div4);
    a.J[2][ANGLE] = -d4 * ddiv4_angle / (div4 * div4);
    out.push_back(a);
  }
  return out;
}

// Pose rows (tip xyz, psi, vel xyz, omega) and their Jacobians for steps 0..max_steps-1.
void pose_table(const ddm_config& c, const ddm_instance& in, std::vector<double>& pose, std::vector<double>& jac) {
  const std::vector<Action> acts = skill_actions(c, in);
  pose.assign((size_t)c.max_steps * 8, 0.0);
  jac.assign((size_t)c.max_steps * 8 * kSkill, 0.0);
  double tip[3] = {in.tip0[0], in.tip0[1], in.tip0[2]}, psi = 0.0;
  double Jtip[3][kSkill] = {{0}}, Jpsi[kSkill] = {0};
  const double inv_n = 1.0 / c.n_sub;
  for (int n = 0; n < c.max_steps; ++n) {
    const size_t t = (size_t)(n / c.n_sub);
    double* row = &pose[(size_t)n * 8];
    double* J = &jac[(size_t)n * 8 * kSkill];
    double vel[3] = {0, 0, 0}, om = 0.0, Jvel[3][kSkill] = {{0}}, Jom[kSkill] = {0};
    if (t < acts.size()) {
      const Action& a = acts[t];
      const int map[3] = {0, 2, 1};                // build axis k takes paper entry map[k]
      for (int k = 0; k < 3; ++k) {
        const double dk = a.d[map[k]] * inv_n;
        tip[k] += dk;
        vel[k] = dk / in.dt;
        for (int j = 0; j < kSkill; ++j) {
          Jtip[k][j] += a.J[map[k]][j] * inv_n;
          Jvel[k][j] = a.J[map[k]][j] * inv_n / in.dt;
        }
      }
      const double dpsi = a.d[3] * inv_n;
      psi += dpsi;
      om = dpsi / in.dt;
      for (int j = 0; j < kSkill; ++j) { Jpsi[j] += a.J[3][j] * inv_n; Jom[j] = a.J[3][j] * inv_n / in.dt; }
    }
    for (int k = 0; k < 3; ++k) { row[k] = tip[k]; row[4 + k] = vel[k]; }
    row[3] = psi;
    row[7] = om;
    for (int j = 0; j < kSkill; ++j) {
      for (int k = 0; k < 3; ++k) { J[k * kSkill + j] = Jtip[k][j]; J[(4 + k) * kSkill + j] = Jvel[k][j]; }
      J[3 * kSkill + j] = Jpsi[j];
      J[7 * kSkill + j] = Jom[j];
    }
  }
}

}  // namespace

// Launch groups timed by ddm_set_timing.
constexpr int kTimingGroups = 10;

struct ddm_ctx {
  ddm_config cfg;
  int n_inst = 0;
  std::vector<ddm_instance> inst;
  Layout L;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  ddm::KCfg kc;
  int prec = 0;
  int64_t steps = 0;             // sub-steps since ddm_init_state
  bool initialised = false;
  bool recorded = false;         // a rollout is recorded
  int64_t rec_k0 = 0, rec_n = 0;
  bool loss_ready = false;
  bool need_sort = true;          // re-bin before the next sub-step
  bool grid_valid = false;        // grid_pre/grid_post and the active set are those of the last sub-step
  // the current particle state and its ids live in one of two buffers each;
  // a binning gathers into the other one and the two swap roles
  size_t cur_off = 0, spare_off = 0, pid_off = 0, pid_spare_off = 0;
  // captured full pass (ddm_pass with use_graph): the graph and the arguments it was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void* g_x0 = nullptr;
  const double *g_target = nullptr, *g_dloss = nullptr;
  double *g_loss = nullptr, *g_grad = nullptr;
  int32_t g_steps = 0;
  size_t g_cur_off = 0, g_spare_off = 0, g_pid_off = 0, g_pid_spare_off = 0;   // buffer roles at the end of the captured pass
  std::vector<char> rec_sorted;   // per recorded step: binned at its start
  // The rollout runs its last checkpoint segments (as many as there are sets
  // of segment buffers) straight into those buffers, the last segment into
  // set 0, the one before into set 1, ...; the reverse pass replays only the
  // others.  rec_first: the first segment so recorded while the buffers still
  // hold them (INT32_MAX: none); rec_tl_of[set]: per-step tile lists.
  int rec_first = INT32_MAX;
  std::vector<std::vector<int>> rec_tl_of;
  // kernel timing
  int32_t timing = 0;             // groups bracketed by timing events (bit g: group g)
  struct Ev { int group; hipEvent_t a, b; };
  std::vector<Ev> events;
  std::vector<hipEvent_t> pool;
  double t_ms[kTimingGroups] = {0};
  int64_t t_n[kTimingGroups] = {0};
  // gradient treatments of the reverse pass and the caller's statistics buffer
  ddm::Treat treat{ddm::kTreatNone, 1e4, 4.0, 1e-6};
  double* stats_dev = nullptr;
  int32_t stats_steps = 0;
  int32_t emd_m = 0;              // target points per instance set by ddm_set_emd_target (0: none)

  template <typename T = char> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  void* cur() const { return at(cur_off); }
  uint32_t* pid() const { return at<uint32_t>(pid_off); }
  // a persistent launch (tile_workgroups > 0) takes its tiles from the queue words
  uint32_t* tile_queue() const { return cfg.tile_workgroups > 0 ? at<uint32_t>(L.tqueue) : nullptr; }
  ddm::TileList tiles() const {
    return ddm::TileList{at<const ddm::TileRec>(L.tiles), at<const uint32_t>(L.tcount), tile_queue()};
  }
  // buffers of sub-step j of segment-buffer set m
  size_t sb(int m) const { return (size_t)m * L.seg_set; }
  void* slot(int m, int j) const { return at(sb(m) + L.seg_state + (size_t)j * L.state_bytes); }
  void* gpre(int m, int j) const { return at(sb(m) + L.seg_grid + (size_t)j * L.rec_bytes); }
  void* tau(int m, int j) const { return at(sb(m) + L.seg_tau + L.tau_bytes * (size_t)j); }
  uint32_t* perm(int m, int j) const { return at<uint32_t>(sb(m) + L.seg_perm + sizeof(uint32_t) * (size_t)L.ntot * j); }
  ddm::TileRec* seg_tile_recs(int m, int j) const {
    return at<ddm::TileRec>(sb(m) + L.seg_tiles + sizeof(ddm::TileRec) * L.max_chunks * j);
  }
  uint32_t* seg_tcount(int m, int j) const { return at<uint32_t>(sb(m) + L.seg_tcount + sizeof(uint32_t) * j); }
  ddm::TileList seg_tiles(int m, int j) const { return ddm::TileList{seg_tile_recs(m, j), seg_tcount(m, j), tile_queue()}; }
  ddm::Staging staging() const { return ddm::Staging{at<void>(L.staging), at<const uint32_t>(L.tslot)}; }
  ddm::ActiveSet active() const {
    return ddm::ActiveSet{at<uint32_t>(L.amask), at<uint32_t>(L.alist), at<uint32_t>(L.acount)};
  }
  uint32_t* seg_alist(int m, int j) const {
    return at<uint32_t>(sb(m) + L.seg_alist + sizeof(uint32_t) * L.total_tiles * j);
  }
  uint32_t* seg_acount(int m, int j) const { return at<uint32_t>(sb(m) + L.seg_acount + sizeof(uint32_t) * j); }
  uint32_t* ckpt_pid(int64_t k) const { return at<uint32_t>(L.ckpt_pid + sizeof(uint32_t) * (size_t)L.ntot * k); }
  ddm::Bufs bufs() const {
    ddm::Bufs b;
    b.inst = at<const ddm::InstDev>(L.inst);
    b.blk_inst = at<const int>(L.blk_inst);
    b.poses = at<const void>(L.poses);
    b.err = at<ddm::DevErr>(L.err);
    b.dpart = cfg.deterministic ? at<double>(L.dpart) : nullptr;
    return b;
  }
  ddm::EmdBufs emdbufs() const {
    ddm::EmdBufs e;
    e.top = at<unsigned long long>(L.emd_top);
    e.own = at<unsigned long long>(L.emd_own);
    e.target = at<double>(L.emd_target);
    e.obs = at<double>(L.emd_obs);
    e.obs_slot = at<int>(L.emd_slot);
    e.n_obs = at<int>(L.emd_nobs);
    e.assign = at<int>(L.emd_assign);
    e.emd = at<double>(L.emd_val);
    return e;
  }
  ddm::LossBufs lossbufs() const {
    ddm::LossBufs l;
    l.hm_bits = at<unsigned long long>(L.hm_bits);
    l.owner = at<unsigned int>(L.owner);
    l.target = at<const double>(L.target);
    l.hm_val = at<double>(L.hm_val);
    l.dldh = at<double>(L.dldh);
    l.region = at<double>(L.region);
    l.dldm = at<double>(L.dldm);
    l.loss = at<double>(L.loss);
    return l;
  }
};

namespace {

ddm_status validate(const ddm_config* c, int32_t n_inst, const ddm_instance* in) {
  if (!c) return fail(DDM_EINVAL, "config is NULL");
  if (c->dim != 2 && c->dim != 3) return fail(DDM_EINVAL, "dim must be 2 or 3");
  if (!is_pow2(c->n_grid) || c->n_grid < 16 || c->n_grid > 256)
    return fail(DDM_EINVAL, "n_grid must be a power of two in [16, 256]");
  if (c->bound < 0 || c->bound > c->n_grid / 4) return fail(DDM_EINVAL, "bound out of [0, n_grid/4]");
  if (c->precision != DDM_F32 && c->precision != DDM_F64) return fail(DDM_EINVAL, "precision must be DDM_F32 or DDM_F64");
  if (c->shovel && c->dim != 3) return fail(DDM_EINVAL, "the shovel needs dim 3");
  if (c->n_sub < 1) return fail(DDM_EINVAL, "n_sub must be >= 1");
  if (!(c->ppc > 0)) return fail(DDM_EINVAL, "ppc must be > 0");
  if (c->hm_res < 1 || c->hm_res > 4096) return fail(DDM_EINVAL, "hm_res out of [1, 4096]");
  if (!(c->hm_size > 0)) return fail(DDM_EINVAL, "hm_size must be > 0");
  if (c->checkpoint_every < 1) return fail(DDM_EINVAL, "checkpoint_every must be >= 1");
  if (c->record_segments < 0) return fail(DDM_EINVAL, "record_segments must be >= 0");
  if (c->max_steps < 1) return fail(DDM_EINVAL, "max_steps must be >= 1");
  if (c->sort_every < 0) return fail(DDM_EINVAL, "sort_every must be >= 0");
  if (c->tile_workgroups < 0 || c->tile_workgroups > (1 << 22)) return fail(DDM_EINVAL, "tile_workgroups out of [0, 2^22]");
  if (c->grid_record_blocks < 0) return fail(DDM_EINVAL, "grid_record_blocks < 0");
  if (c->deterministic != 0 && c->deterministic != 1) return fail(DDM_EINVAL, "deterministic must be 0 or 1");
  if (c->w_emd != 0.0 && c->dim != 3) return fail(DDM_EINVAL, "the EMD term needs dim 3");
  if (c->w_emd != 0.0 && c->hm_res * c->hm_res > ddm::kEmdMaxPoints)
    return fail(DDM_EINVAL, "the EMD term needs hm_res^2 <= 4096");
  if (!std::isfinite(c->w_emd)) return fail(DDM_EINVAL, "w_emd must be finite");
  if (c->shovel && !(c->v_lin > 0 && c->v_ang > 0 && c->d_lift > 0 && c->contact_skin >= 0 && c->shovel_mu >= 0))
    return fail(DDM_EINVAL, "shovel speeds, lift, skin and friction must be positive");
  if (n_inst < 1 || !in) return fail(DDM_EINVAL, "need at least one instance");
  int64_t nodes = 1;
  for (int a = 0; a < c->dim; ++a) nodes *= c->n_grid;
  if ((double)nodes * n_inst * ddm::kNodeVals > 9.0e18) return fail(DDM_EINVAL, "grid too large");
  int64_t ntot = 0;
  for (int i = 0; i < n_inst; ++i) {
    const ddm_instance& s = in[i];
    char buf[160];
    auto bad = [&](const char* what) {
      std::snprintf(buf, sizeof(buf), "instance %d: %s", i, what);
      return fail(DDM_EINVAL, buf);
    };
    if (s.n_particles <= 0) return bad("n_particles must be > 0");
    if (s.n_particles > 0x7FFFFFFF) return bad("n_particles too large");
    if (!(s.E > 0)) return bad("E must be > 0");
    if (!(s.nu > -1.0 && s.nu < 0.5)) return bad("nu must be in (-1, 0.5)");
    if (!(s.phi_deg > 0 && s.phi_deg < 90)) return bad("phi_deg must be in (0, 90)");
    if (!(s.rho > 0)) return bad("rho must be > 0");
    if (!(s.cohesion >= 0)) return bad("cohesion must be >= 0");
    if (!(s.dt > 0)) return bad("dt must be > 0");
    if (c->shovel && !(s.depth >= 0 && s.push >= 0)) return bad("skill depth and push must be >= 0");
    ntot += pad_up(s.n_particles, ddm::kBlock);
  }
  if (ntot > ((int64_t)1 << 31)) return fail(DDM_EINVAL, "too many particles in total");
  return DDM_OK;
}

template <typename T>
void to_prec(const std::vector<double>& src, std::vector<char>& out) {
  out.resize(src.size() * sizeof(T));
  T* d = reinterpret_cast<T*>(out.data());
  for (size_t i = 0; i < src.size(); ++i) d[i] = (T)src[i];
}

ddm_status launch_status() { return hip_check(hipGetLastError(), "kernel launch"); }

hipEvent_t take_event(ddm_ctx* x) {
  if (!x->pool.empty()) { hipEvent_t e = x->pool.back(); x->pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets a launch group with events when timing selects its group.
struct Timed {
  ddm_ctx* x;
  int group;
  hipEvent_t a = nullptr;
  Timed(ddm_ctx* x_, int g) : x(x_), group(g) {
    if (((x->timing >> group) & 1) && (a = take_event(x))) (void)hipEventRecord(a, x->stream);
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = take_event(x);
    if (!b) return;
    (void)hipEventRecord(b, x->stream);
    x->events.push_back(ddm_ctx::Ev{group, a, b});
  }
};

void resolve_events(ddm_ctx* x) {
  for (const auto& e : x->events) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) { x->t_ms[e.group] += ms; x->t_n[e.group] += 1; }
    x->pool.push_back(e.a);
    x->pool.push_back(e.b);
  }
  x->events.clear();
}

// Bins the particles of state `src` into `dst` (another buffer): exact cell
// keys, stable radix sort by (instance, tile, cell), gather of the state rows
// (and ids, when given) into sorted order, the occupied-tile list with each
// tile's staging record, and the active node blocks.  When perm_out / tiles_out are given the
// permutation and the tile list are also stored there (for the reverse pass).
ddm_status bin_state(ddm_ctx* x, const void* src, void* dst, const uint32_t* pid_src, uint32_t* pid_dst,
                     uint32_t* perm_out, ddm::TileRec* tiles_out, uint32_t* tcount_out) {
  Timed tm(x, 3);
  const Layout& L = x->L;
  hipStream_t st = x->stream;
  uint32_t* keys[2] = {x->at<uint32_t>(L.keys0), x->at<uint32_t>(L.keys1)};
  uint32_t* vals[2] = {x->at<uint32_t>(L.vals0), x->at<uint32_t>(L.vals1)};
  int r = 0;
  if (x->kc.det) {
    // deterministic mode: a cell's particles in id order, whatever their slot
    // order before (a stable sort by id, then the stable sort by cell)
    if (!pid_src) return fail(DDM_ESTATE, "binning without particle ids in the deterministic mode");
    ddm::launch_pid_keys(pid_src, keys[0], vals[0], L.ntot, st);
    const int r1 = ddm::radix_sort(keys, vals, L.ntot, (uint32_t)L.ntot, x->at<uint32_t>(L.hist),
                                   x->at<uint32_t>(L.sums), st);
    uint32_t* k2[2] = {keys[1 - r1], keys[r1]};
    uint32_t* v2[2] = {vals[1 - r1], vals[r1]};
    ddm::launch_keys(x->prec, x->kc, x->bufs(), (int)L.nblk, src, k2[0], v2[0], st, vals[r1]);
    const int r2 = ddm::radix_sort(k2, v2, L.ntot, L.max_key, x->at<uint32_t>(L.hist), x->at<uint32_t>(L.sums), st);
    r = k2[r2] == keys[0] ? 0 : 1;
  } else {
    ddm::launch_keys(x->prec, x->kc, x->bufs(), (int)L.nblk, src, keys[0], vals[0], st);
    r = ddm::radix_sort(keys, vals, L.ntot, L.max_key, x->at<uint32_t>(L.hist), x->at<uint32_t>(L.sums), st);
  }
  ddm::launch_gather(L.esz, src, dst, vals[r], L.rows, L.ntot, pid_src, pid_dst, st);
  ddm::launch_tile_list(x->kc, keys[r], x->at<uint32_t>(L.tstart), x->at<uint32_t>(L.tend), x->at<ddm::TileRec>(L.tiles),
                        x->at<uint32_t>(L.tcount), x->at<uint32_t>(L.tslot), x->at<uint32_t>(L.tbucket), st);
  ddm::launch_active_set(x->kc, x->tiles(), x->active(), st);
  if (perm_out) DDM_HIP(hipMemcpyAsync(perm_out, vals[r], sizeof(uint32_t) * L.ntot, hipMemcpyDeviceToDevice, st));
  if (tiles_out) {
    DDM_HIP(hipMemcpyAsync(tiles_out, x->at(L.tiles), sizeof(ddm::TileRec) * L.max_chunks, hipMemcpyDeviceToDevice, st));
    DDM_HIP(hipMemcpyAsync(tcount_out, x->at(L.tcount), sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
  }
  return launch_status();
}

// Bins the current state into the spare buffers and swaps the roles.
ddm_status bin_current(ddm_ctx* x) {
  const ddm_status s = bin_state(x, x->cur(), x->at(x->spare_off), x->pid(), x->at<uint32_t>(x->pid_spare_off), nullptr,
                                 nullptr, nullptr);
  std::swap(x->cur_off, x->spare_off);
  std::swap(x->pid_off, x->pid_spare_off);
  return s;
}

// Workgroups of P2G: the configured persistent count, or about one per
// occupied tile.
int tile_workgroups(const ddm_ctx* x) {
  return x->cfg.tile_workgroups > 0 ? (int)x->cfg.tile_workgroups : x->L.nwg;
}

// One forward sub-step from st_in to st_out (may alias) with the given tile
// list; grids given.  The reverse pass also keeps the stress (tau_out) and the
// active blocks of the sub-step (list_out, count_out).
ddm_status forward_step(ddm_ctx* x, int64_t step, const ddm::TileList& tl, const void* st_in, void* st_out,
                        void* gpre, void* gpost, void* tau_out = nullptr, uint32_t* list_out = nullptr,
                        uint32_t* count_out = nullptr) {
  const ddm::Bufs b = x->bufs();
  const ddm::Staging stg = x->staging();
  const ddm::ActiveSet act = x->active();
  void* gout = x->at(x->L.gout);
  { Timed t(x, 0); ddm::launch_p2g(x->prec, x->kc, b, tl, tile_workgroups(x), st_in, st_out, stg, gout, act, tau_out, x->stream); }
  // a recorded sub-step (list_out given) writes its pre-update grid as a record in active-list order
  { Timed t(x, 1); ddm::launch_grid_update(x->prec, x->kc, b, (int)step, stg, gout, act, gpre,
                                           list_out ? x->L.rec_items : -1, gpost, list_out, count_out, x->stream); }
  { Timed t(x, 2); ddm::launch_g2p(x->prec, x->kc, b, (int)x->L.nblk, (int)step, st_in, st_out, gpost, x->stream); }
  return launch_status();
}

// The deterministic mode bins before every sub-step (a cell's particles then
// form one run of the tile kernels' scatter).
bool sort_due(const ddm_ctx* x, int64_t step) {
  const int R = x->cfg.sort_every;
  return x->need_sort || x->cfg.deterministic || (R > 0 && step % R == 0);
}

// Runs `len` sub-steps from step k_first into the segment buffers as the
// reverse pass needs them: the state before step j in slot j (the state after
// the last in slot len), its grids, stress, binning permutation, tile list and
// active blocks.  bins[j] says whether step j bins first (from `src` for
// j = 0, else from the spare state buffer that step j - 1 wrote).  With
// move_pid the particle ids follow each binning (the forward pass); the
// replay of the reverse pass leaves them alone.  tl_of[j]: the slot whose
// tile list step j uses.
ddm_status run_segment(ddm_ctx* x, int m, int64_t k_first, int len, const void* src, const char* bins,
                       bool move_pid, std::vector<int>& tl_of, const uint32_t* replay_pid = nullptr) {
  void* spare = x->at(x->spare_off);
  tl_of.assign((size_t)len, 0);
  int last = 0;
  // a replay in the deterministic mode carries the ids of its checkpoint
  // through its binnings in a pair of its own
  uint32_t* rp[2] = {x->at<uint32_t>(x->L.rpid0), x->at<uint32_t>(x->L.rpid1)};
  const uint32_t* rpid_cur = replay_pid;
  int rsel = 0;
  for (int j = 0; j < len; ++j) {
    if (bins[j]) {
      const uint32_t* pin = move_pid ? x->pid() : rpid_cur;
      uint32_t* pout = move_pid ? x->at<uint32_t>(x->pid_spare_off) : (rpid_cur ? rp[rsel] : nullptr);
      const ddm_status s = bin_state(x, j == 0 ? src : spare, x->slot(m, j), pin, pout, x->perm(m, j),
                                     x->seg_tile_recs(m, j), x->seg_tcount(m, j));
      if (s != DDM_OK) return s;
      if (move_pid) std::swap(x->pid_off, x->pid_spare_off);
      else if (rpid_cur) { rpid_cur = rp[rsel]; rsel = 1 - rsel; }
      last = j;
    } else if (j == 0) {
      DDM_HIP(hipMemcpyAsync(x->slot(m, 0), src, x->L.state_bytes, hipMemcpyDeviceToDevice, x->stream));
    }
    tl_of[j] = last;
    const bool next_bins = j + 1 < len && bins[j + 1];
    const ddm_status s = forward_step(x, k_first + j, x->seg_tiles(m, last), x->slot(m, j),
                                      next_bins ? spare : x->slot(m, j + 1), x->gpre(m, j), x->at(x->L.grid_post),
                                      x->tau(m, j), x->seg_alist(m, j), x->seg_acount(m, j));
    if (s != DDM_OK) return s;
  }
  return DDM_OK;
}

// Per-instance constants (Lame constants from (E, nu), alpha_f and the
// cohesion shift from the friction angle, particle mass and volume, and their
// derivatives for the final chain rule), the block-to-instance map, and the
// pose table with its Jacobian; uploaded with synchronous copies.
// Kernel configuration of a context (or of a context-free call) with
// n_inst instances and ntot padded particle slots.
ddm::KCfg make_kcfg(const ddm_config& c, int n_inst, int64_t ntot) {
  ddm::KCfg k;
  k.dim = c.dim; k.n = c.n_grid; k.bound = c.bound; k.shovel = c.shovel;
  k.pcontact = c.particle_contact != 0 ? 1 : 0;
  k.nlog2 = 0;
  while ((1 << k.nlog2) < c.n_grid) ++k.nlog2;
  k.hm_res = c.hm_res; k.region_sign = c.region_sign >= 0 ? 1 : -1; k.n_inst = n_inst;
  k.max_steps = c.max_steps;
  k.nodes = 1;
  for (int a = 0; a < c.dim; ++a) k.nodes *= c.n_grid;
  k.ntot = ntot;
  k.dx = 1.0 / c.n_grid; k.inv_dx = (double)c.n_grid; k.gravity = c.gravity;
  k.skin = c.contact_skin; k.mu_b = c.shovel_mu;
  for (int a = 0; a < 3; ++a) k.half[a] = c.shovel_half[a];
  k.hm_ox = c.hm_origin[0]; k.hm_oz = c.hm_origin[1]; k.hm_pix = c.hm_size / c.hm_res;
  k.hm_off = c.hm_offset; k.region_depth = c.region_depth;
  k.w_hm = c.w_hm; k.w_mass = c.w_mass; k.m_target = c.m_target; k.m_ref = c.m_ref;
  k.w_emd = c.w_emd;
  k.det = c.deterministic ? 1 : 0;
  return k;
}

// Device constants of instance i: Lame constants, alpha_f and the cohesion
// shift (Sec. III-A, Eq. DP), particle mass and volume, the chain to
// (E, nu, phi_deg), its first padded slot `off` and its grid offset.
ddm::InstDev make_instdev(const ddm_config& c, const ddm_instance& s, int i, int64_t off, int64_t nodes) {
  ddm::InstDev d;
  const double dxd = std::pow(1.0 / c.n_grid, c.dim);
  const double E = s.E, nu = s.nu, ph = s.phi_deg * kPi / 180.0, sp = std::sin(ph), cp = std::cos(ph);
  d.mu = E / (2.0 * (1.0 + nu));
  d.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double r23 = std::sqrt(2.0 / 3.0);
  d.alpha = r23 * 2.0 * sp / (3.0 - sp);
  d.kc = r23 * 6.0 * s.cohesion * cp / (3.0 - sp);
  d.Vp = dxd / c.ppc;
  d.mp = s.rho * d.Vp;
  d.dt = s.dt;
  d.dmu_dE = 1.0 / (2.0 * (1.0 + nu));
  d.dmu_dnu = -E / (2.0 * (1.0 + nu) * (1.0 + nu));
  const double den = (1.0 + nu) * (1.0 - 2.0 * nu);
  d.dlam_dE = nu / den;
  d.dlam_dnu = E * (1.0 + 2.0 * nu * nu) / (den * den);
  const double rad = kPi / 180.0;
  d.dal_dphi = r23 * 6.0 * cp / ((3.0 - sp) * (3.0 - sp)) * rad;
  d.dkc_dphi = r23 * 6.0 * s.cohesion * (1.0 - 3.0 * sp) / ((3.0 - sp) * (3.0 - sp)) * rad;
  d.off = off;
  d.n = s.n_particles;
  d.goff = (int64_t)i * nodes;
  for (int a = 0; a < 3; ++a) d.tip0[a] = s.tip0[a];
  return d;
}

ddm_status upload_instances(ddm_ctx* x, const ddm_instance* inst) {
  const ddm_config* cfg = &x->cfg;
  const Layout& L = x->L;
  const int n_inst = x->n_inst;
  const ddm::KCfg& k = x->kc;
  ddm_status s = DDM_OK;
  std::vector<ddm::InstDev> dev(n_inst);
  std::vector<int> blk((size_t)L.nblk);
  int64_t off = 0;
  for (int i = 0; i < n_inst; ++i) {
    const ddm_instance& s = inst[i];
    dev[i] = make_instdev(*cfg, s, i, off, k.nodes);
    const int64_t np = pad_up(s.n_particles, ddm::kBlock);
    for (int64_t bI = off / ddm::kBlock; bI < (off + np) / ddm::kBlock; ++bI) blk[(size_t)bI] = i;
    off += np;
  }
  const size_t js = (size_t)8 * kSkill;      // pose Jacobian values per sub-step
  std::vector<double> poses((size_t)n_inst * cfg->max_steps * 8, 0.0), jac((size_t)n_inst * cfg->max_steps * js, 0.0);
  if (cfg->shovel) {
    for (int i = 0; i < n_inst; ++i) {
      std::vector<double> p, j;
      pose_table(*cfg, inst[i], p, j);
      std::copy(p.begin(), p.end(), poses.begin() + (size_t)i * cfg->max_steps * 8);
      std::copy(j.begin(), j.end(), jac.begin() + (size_t)i * cfg->max_steps * js);
    }
  }
  // device rows: the 8 pose values and sin / cos of the blade angle
  std::vector<double> prow((size_t)n_inst * cfg->max_steps * ddm::kPoseVals, 0.0);
  for (size_t r = 0; r < (size_t)n_inst * cfg->max_steps; ++r) {
    std::copy(poses.begin() + r * 8, poses.begin() + r * 8 + 8, prow.begin() + r * ddm::kPoseVals);
    prow[r * ddm::kPoseVals + 8] = std::sin(poses[r * 8 + 3]);
    prow[r * ddm::kPoseVals + 9] = std::cos(poses[r * 8 + 3]);
  }
  std::vector<char> poses_t;
  if (x->prec) to_prec<double>(prow, poses_t); else to_prec<float>(prow, poses_t);
  // Host staging arrays are copied synchronously so the caller's memory is free on return.
  s = hip_check(hipMemcpy(x->at(L.inst), dev.data(), sizeof(ddm::InstDev) * n_inst, hipMemcpyHostToDevice), "upload instances");
  if (s == DDM_OK) s = hip_check(hipMemcpy(x->at(L.blk_inst), blk.data(), sizeof(int) * blk.size(), hipMemcpyHostToDevice), "upload block map");
  if (s == DDM_OK) s = hip_check(hipMemcpy(x->at(L.poses), poses_t.data(), poses_t.size(), hipMemcpyHostToDevice), "upload poses");
  if (s == DDM_OK) s = hip_check(hipMemcpy(x->at(L.pose_jac), jac.data(), jac.size() * sizeof(double), hipMemcpyHostToDevice), "upload pose Jacobian");
  return s;
}

}  // namespace

extern "C" {

const char* ddm_status_str(ddm_status s) {
  switch (s) {
    case DDM_OK: return "ok";
    case DDM_EINVAL: return "invalid argument";
    case DDM_ENOMEM: return "workspace too small";
    case DDM_EDEVICE: return "device error";
    case DDM_ENAN: return "NaN or Inf in the state";
    case DDM_EDOMAIN: return "particle stencil left the grid";
    case DDM_ESTATE: return "call out of order";
  }
  return "unknown status";
}

const char* ddm_last_error(void) { return g_last_error.c_str(); }

ddm_status ddm_validate_config(const ddm_config* cfg, int32_t n_inst, const ddm_instance* inst, char* msg,
                               size_t msg_len) {
  const ddm_status s = validate(cfg, n_inst, inst);
  if (msg && msg_len) {
    const std::string& m = s == DDM_OK ? std::string() : g_last_error;
    std::snprintf(msg, msg_len, "%s", m.c_str());
  }
  return s;
}

ddm_status ddm_skill_pose_table(const ddm_config* cfg, const ddm_instance* inst, int32_t n_steps,
                                double* pose_out, double* jac_out) {
  if (!cfg || !inst || !pose_out) return fail(DDM_EINVAL, "NULL argument");
  if (n_steps < 1) return fail(DDM_EINVAL, "n_steps must be >= 1");
  ddm_config c = *cfg;
  c.max_steps = n_steps;
  std::vector<double> p, j;
  pose_table(c, *inst, p, j);
  std::copy(p.begin(), p.end(), pose_out);
  if (jac_out) std::copy(j.begin(), j.end(), jac_out);
  return DDM_OK;
}

ddm_status ddm_workspace_query(const ddm_config* cfg, int32_t n_inst, const ddm_instance* inst, ddm_sizes* out) {
  const ddm_status s = validate(cfg, n_inst, inst);
  if (s != DDM_OK) return s;
  if (!out) return fail(DDM_EINVAL, "out is NULL");
  const Layout L = make_layout(*cfg, n_inst, inst);
  out->workspace_bytes = L.total;
  out->state_bytes = L.state_bytes;
  out->padded_particles = L.ntot;
  return DDM_OK;
}

ddm_status ddm_create(const ddm_config* cfg, int32_t n_inst, const ddm_instance* inst, void* workspace,
                      size_t workspace_bytes, void* stream, ddm_ctx** out) {
  if (!out) return fail(DDM_EINVAL, "out is NULL");
  *out = nullptr;
  ddm_status s = validate(cfg, n_inst, inst);
  if (s != DDM_OK) return s;
  const Layout L = make_layout(*cfg, n_inst, inst);
  if (!workspace) return fail(DDM_EINVAL, "workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(DDM_EINVAL, "workspace must be 256-byte aligned");
  if (workspace_bytes < L.total)
    return fail(DDM_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes, got " +
                                std::to_string(workspace_bytes));
  ddm_ctx* x = new ddm_ctx();
  x->cfg = *cfg;
  x->n_inst = n_inst;
  x->inst.assign(inst, inst + n_inst);
  x->L = L;
  x->cur_off = L.cur;
  x->spare_off = L.scratch;
  x->pid_off = L.pid;
  x->pid_spare_off = L.pid_tmp;
  x->ws = static_cast<char*>(workspace);
  x->stream = static_cast<hipStream_t>(stream);
  x->prec = cfg->precision == DDM_F64 ? 1 : 0;
  x->kc = make_kcfg(*cfg, n_inst, L.ntot);

  s = upload_instances(x, inst);
  if (s == DDM_OK) s = hip_check(hipMemset(x->at(L.err), 0, sizeof(ddm::DevErr)), "clear error word");
  if (s == DDM_OK) s = hip_check(hipMemset(x->at(L.tqueue), 0, 2 * sizeof(uint32_t)), "clear tile queue");
  if (s == DDM_OK && cfg->deterministic)
    s = hip_check(hipMemset(x->at(L.dpart), 0, sizeof(double) * ddm::kDetVals * (size_t)std::max(L.nblk, L.total_tiles)),
                  "clear deterministic partials");
  if (s != DDM_OK) { delete x; return s; }
  *out = x;
  return DDM_OK;
}

ddm_status ddm_set_instances(ddm_ctx* x, int32_t n_inst, const ddm_instance* inst) {
  if (!x || !inst) return fail(DDM_EINVAL, "NULL argument");
  if (n_inst != x->n_inst) return fail(DDM_EINVAL, "the instance count is fixed at ddm_create");
  for (int i = 0; i < n_inst; ++i)
    if (inst[i].n_particles != x->inst[(size_t)i].n_particles)
      return fail(DDM_EINVAL, "instance " + std::to_string(i) + ": the particle count is fixed at ddm_create");
  const ddm_status v = validate(&x->cfg, n_inst, inst);
  if (v != DDM_OK) return v;
  // kernels in flight may still read the old constants
  DDM_HIP(hipStreamSynchronize(x->stream));
  x->inst.assign(inst, inst + n_inst);
  const ddm_status s = upload_instances(x, inst);
  if (s != DDM_OK) return s;
  x->recorded = false;
  x->loss_ready = false;
  return DDM_OK;
}

ddm_status ddm_init_state(ddm_ctx* x, const void* x0_dev) {
  if (!x || !x0_dev) return fail(DDM_EINVAL, "NULL argument");
  ddm::launch_init_state(x->prec, x->kc, x->bufs(), (int)x->L.nblk, x0_dev, x->cur(), x->pid(),
                         x->stream);
  // fill kernels rather than memset nodes, so that the call can be captured in a graph
  ddm::launch_fill_zero(x->at(x->L.err), sizeof(ddm::DevErr) / 4, 4, x->stream);
  ddm::launch_fill_zero(x->at(x->L.gout), (int64_t)(x->L.grid_bytes / 4), 4, x->stream);
  x->grid_valid = false;
  x->steps = 0;
  x->initialised = true;
  x->recorded = false;
  x->loss_ready = false;
  x->need_sort = true;
  return launch_status();
}

ddm_status ddm_step(ddm_ctx* x, int32_t n_steps) {
  Phase phase("ddm_step");
  if (!x) return fail(DDM_EINVAL, "NULL context");
  if (!x->initialised) return fail(DDM_ESTATE, "ddm_init_state first");
  if (n_steps < 0) return fail(DDM_EINVAL, "n_steps < 0");
  if (x->cfg.shovel && x->steps + n_steps > x->cfg.max_steps)
    return fail(DDM_EINVAL, "steps beyond max_steps (the pose table length)");
  for (int i = 0; i < n_steps; ++i) {
    if (sort_due(x, x->steps)) {
      const ddm_status s = bin_current(x);
      if (s != DDM_OK) return s;
      x->need_sort = false;
    }
    const ddm_status s = forward_step(x, x->steps, x->tiles(), x->cur(), x->cur(), x->at(x->L.grid_pre),
                                      x->at(x->L.grid_post));
    if (s != DDM_OK) return s;
    ++x->steps;
    x->grid_valid = true;
  }
  x->recorded = false;
  x->loss_ready = false;
  return DDM_OK;
}

ddm_status ddm_rollout(ddm_ctx* x, int32_t n_steps) {
  Phase phase("ddm_rollout");
  if (!x) return fail(DDM_EINVAL, "NULL context");
  if (!x->initialised) return fail(DDM_ESTATE, "ddm_init_state first");
  if (n_steps < 1) return fail(DDM_EINVAL, "n_steps must be >= 1");
  if (x->steps + n_steps > x->cfg.max_steps) return fail(DDM_EINVAL, "rollout longer than max_steps");
  const int K = x->L.K;
  const int64_t k0 = x->steps;
  const Layout& L = x->L;
  x->rec_sorted.assign((size_t)n_steps, 0);
  x->rec_first = INT32_MAX;
  // sub-steps before the recorded checkpoint segments; those go straight into
  // the segment buffers, so the reverse pass does not replay them
  const int nseg = (n_steps + K - 1) / K;
  const int first_rec = nseg - std::min(L.M, nseg);
  const int64_t s_rec = (int64_t)first_rec * K;
  {
  Phase plain("unrecorded sub-steps", s_rec > 0);
  for (int i = 0; i < s_rec; ++i) {
    // Checkpoints hold the state before the binning of their step; every
    // checkpointed step re-bins, so a replayed segment needs nothing older.
    if (i % K == 0) {
      DDM_HIP(hipMemcpyAsync(x->at(x->L.ckpt + (size_t)(i / K) * x->L.state_bytes), x->cur(), x->L.state_bytes,
                             hipMemcpyDeviceToDevice, x->stream));
      if (x->kc.det)
        DDM_HIP(hipMemcpyAsync(x->ckpt_pid(i / K), x->pid(), sizeof(uint32_t) * L.ntot, hipMemcpyDeviceToDevice,
                               x->stream));
      x->need_sort = true;
    }
    if (sort_due(x, k0 + i)) {
      const ddm_status s = bin_current(x);
      if (s != DDM_OK) return s;
      x->need_sort = false;
      x->rec_sorted[(size_t)i] = 1;
    }
    const ddm_status s = forward_step(x, k0 + i, x->tiles(), x->cur(), x->cur(), x->at(x->L.grid_pre),
                                      x->at(x->L.grid_post));
    if (s != DDM_OK) return s;
    ++x->steps;
    x->grid_valid = true;
  }
  }
  x->rec_tl_of.assign((size_t)L.M, std::vector<int>());
  const void* src = x->cur();
  int m = 0, len = 0;
  for (int seg = first_rec; seg < nseg; ++seg) {
    const int64_t s0 = (int64_t)seg * K;
    m = nseg - 1 - seg;
    len = (int)std::min<int64_t>(K, n_steps - s0);
    // the checkpoint, for a reverse pass that has to replay the segment after all
    DDM_HIP(hipMemcpyAsync(x->at(L.ckpt + (size_t)seg * L.state_bytes), src, L.state_bytes, hipMemcpyDeviceToDevice,
                           x->stream));
    if (x->kc.det)
      DDM_HIP(hipMemcpyAsync(x->ckpt_pid(seg), x->pid(), sizeof(uint32_t) * L.ntot, hipMemcpyDeviceToDevice, x->stream));
    // the forward's binning decisions: the first step of a segment, then every
    // sort_every steps (every step in the deterministic mode)
    const int R = x->cfg.sort_every;
    for (int j = 0; j < len; ++j)
      x->rec_sorted[(size_t)(s0 + j)] = j == 0 || x->kc.det || (R > 0 && (k0 + s0 + j) % R == 0);
    Phase record("recorded segment");
    const ddm_status s = run_segment(x, m, k0 + s0, len, src, &x->rec_sorted[(size_t)s0], true, x->rec_tl_of[(size_t)m]);
    if (s != DDM_OK) return s;
    src = x->slot(m, len);
    x->steps += len;
  }
  // the final state, its grids and its binning become the current ones
  DDM_HIP(hipMemcpyAsync(x->cur(), src, L.state_bytes, hipMemcpyDeviceToDevice, x->stream));
  // (the post-update grid of the last sub-step is in grid_post already and is
  // rebuilt with the same values; the dense pre-update grid comes from its record)
  ddm::launch_grid_post_from_pre(x->prec, x->kc, x->bufs(), (int)(x->steps - 1), x->seg_alist(m, len - 1),
                                 x->seg_acount(m, len - 1), x->gpre(m, len - 1), L.rec_items, x->at(L.grid_post),
                                 x->at(L.grid_pre), x->stream);
  x->need_sort = false;
  x->grid_valid = true;
  x->rec_first = first_rec;
  x->recorded = true;
  x->rec_k0 = k0;
  x->rec_n = n_steps;
  x->loss_ready = false;
  return DDM_OK;
}

ddm_status ddm_loss(ddm_ctx* x, const double* target_hm_dev, double* loss_dev) {
  Phase phase("ddm_loss");
  if (!x || !target_hm_dev || !loss_dev) return fail(DDM_EINVAL, "NULL argument");
  if (!x->initialised) return fail(DDM_ESTATE, "ddm_init_state first");
  const int npix = x->cfg.dim == 3 ? x->cfg.hm_res * x->cfg.hm_res : x->cfg.hm_res;
  DDM_HIP(hipMemcpyAsync(x->at(x->L.target), target_hm_dev, sizeof(double) * (size_t)x->n_inst * npix,
                         hipMemcpyDeviceToDevice, x->stream));
  if (x->cfg.w_emd != 0.0 && x->emd_m == 0) return fail(DDM_ESTATE, "w_emd != 0 needs ddm_set_emd_target");
  {
    Timed t(x, 8);
    ddm::launch_loss(x->prec, x->kc, x->bufs(), (int)x->L.nblk, x->cur(), x->pid(),
                     (int)x->steps - 1, x->lossbufs(), x->stream);
    if (x->cfg.w_emd != 0.0)
      ddm::launch_emd(x->prec, x->kc, x->bufs(), (int)x->L.nblk, x->cur(), x->pid(), x->emdbufs(), x->emd_m,
                      x->cfg.w_emd, x->at<double>(x->L.loss), x->stream);
  }
  DDM_HIP(hipMemcpyAsync(loss_dev, x->at(x->L.loss), sizeof(double) * x->n_inst, hipMemcpyDeviceToDevice, x->stream));
  x->loss_ready = x->recorded && x->steps == x->rec_k0 + x->rec_n;
  return launch_status();
}

ddm_status ddm_set_emd_target(ddm_ctx* x, const double* points_dev, int32_t m) {
  if (!x || !points_dev) return fail(DDM_EINVAL, "NULL argument");
  if (x->cfg.dim != 3) return fail(DDM_EINVAL, "the EMD term needs dim 3");
  if (x->cfg.w_emd == 0.0) return fail(DDM_EINVAL, "w_emd is 0: the workspace holds no EMD buffers");
  const int npix = x->cfg.hm_res * x->cfg.hm_res;
  if (m < 1 || m > npix) return fail(DDM_EINVAL, "m outside [1, hm_res^2]");
  // [n_inst][m][3] into the workspace's [n_inst][hm_res^2][3]
  DDM_HIP(hipMemcpy2DAsync(x->at(x->L.emd_target), sizeof(double) * 3 * npix, points_dev, sizeof(double) * 3 * m,
                           sizeof(double) * 3 * m, x->n_inst, hipMemcpyDeviceToDevice, x->stream));
  x->emd_m = m;
  return DDM_OK;
}

namespace {

// Gradient treatment of one group of adjoint vectors (Sec. III-E): the
// particle state (grid == false) or the nodes of the listed active blocks of
// one grid buffer.
struct TreatTarget {
  bool grid;
  void* g;                        // adjoint state or grid buffer
  const uint32_t* list = nullptr;
  const uint32_t* count = nullptr;
  int var = 0;                    // first grid variable
  bool with_mass = false;
};

void treat_vectors(ddm_ctx* x, bool record, const TreatTarget& t) {
  unsigned long long* acc = x->at<unsigned long long>(x->L.treat_acc);
  const ddm::Bufs b = x->bufs();
  if (t.grid)
    ddm::launch_treat_grid(x->prec, x->kc, b, t.list, t.count, t.g, t.var, t.with_mass, x->treat, record, acc, x->stream);
  else
    ddm::launch_treat_particles(x->prec, x->kc, b, (int)x->L.nblk, t.g, x->treat, record, acc, x->stream);
}

}  // namespace

ddm_status ddm_backward(ddm_ctx* x, const double* dloss_dev, double* grad_dev) {
  Phase phase("ddm_backward");
  if (!x || !dloss_dev || !grad_dev) return fail(DDM_EINVAL, "NULL argument");
  if (!x->recorded || !x->loss_ready) return fail(DDM_ESTATE, "ddm_backward needs ddm_rollout then ddm_loss");
  const Layout& L = x->L;
  const ddm::Bufs b = x->bufs();
  const int esz = x->prec ? 8 : 4;
  hipStream_t st = x->stream;
  ddm::launch_fill_zero(x->at(L.pacc), (int64_t)8 * x->n_inst, 8, st);
  ddm::launch_fill_zero(x->at(L.pose_bar), (int64_t)8 * x->n_inst * x->cfg.max_steps, 8, st);
  // the v-bar grid starts at zero; each grid adjoint step clears what it read
  { Timed t(x, 7); ddm::launch_fill_zero(x->at(L.gvb), (int64_t)L.grid_bytes / esz, esz, st); }
  const int64_t stat_vals = (int64_t)x->n_inst * ddm::kTreatVars * 6;
  if (x->stats_dev) ddm::launch_fill_zero(x->stats_dev, stat_vals * x->stats_steps, 8, st);
  unsigned long long* acc = x->at<unsigned long long>(L.treat_acc);
  void* adj[2] = {x->at(L.adj0), x->at(L.adj1)};
  int cur = 0;
  ddm::launch_loss_seed(x->prec, x->kc, b, (int)L.nblk, x->cur(), x->pid(), (int)x->steps - 1,
                        x->lossbufs(), adj[cur], x->at<double>(L.pacc), st);
  if (x->cfg.w_emd != 0.0) ddm::launch_emd_seed(x->prec, x->kc, b, x->emdbufs(), x->cfg.w_emd, adj[cur], st);
  const int K = L.K;
  const int64_t n = x->rec_n, k0 = x->rec_k0;
  const int nseg = (int)((n + K - 1) / K);
  const int have = x->rec_first;   // segments the rollout left in the buffers
  x->rec_first = INT32_MAX;        // the replays below overwrite them
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int64_t s0 = (int64_t)seg * K;
    const int len = (int)std::min<int64_t>(K, n - s0);
    // A segment the rollout recorded is in buffer set nseg - 1 - seg.  The
    // others are replayed into set 0 (whose segment, the last, is done by
    // then): same binning steps as the recorded forward pass, the first from
    // the checkpoint.
    const int m = seg >= have ? nseg - 1 - seg : 0;
    std::vector<int> tl_of;
    if (seg >= have) {
      tl_of = x->rec_tl_of[(size_t)m];
    } else {
      Phase replay("replay segment");
      const ddm_status s = run_segment(x, 0, k0 + s0, len, x->at(L.ckpt + (size_t)seg * L.state_bytes),
                                       &x->rec_sorted[(size_t)s0], false, tl_of,
                                       x->kc.det ? x->ckpt_pid(seg) : nullptr);
      if (s != DDM_OK) return s;
    }
    auto slot = [&](int j) { return x->slot(m, j); };
    auto gpre = [&](int j) { return x->gpre(m, j); };
    // post-update grid of the sub-step being reversed, rebuilt into grid_post
    auto gpost = [&](int) { return x->at(L.grid_post); };
    auto perm = [&](int j) { return x->perm(m, j); };
    auto tau = [&](int j) { return x->tau(m, j); };
    Phase reverse("reverse segment");
    for (int j = len - 1; j >= 0; --j) {
      const ddm::TileList tl = x->seg_tiles(m, tl_of[j]);
      const int64_t k = k0 + s0 + j;
      const bool rec = x->stats_dev && k < x->stats_steps;
      const bool treat = rec || x->treat.mode != ddm::kTreatNone;
      const bool reduce = rec || x->treat.mode == ddm::kTreatScale || x->treat.mode == ddm::kTreatNorm;
      if (reduce) { Timed t(x, 9); ddm::launch_fill_zero(acc, (int64_t)ddm::treat_acc_words(x->n_inst), 8, st); }
      { Timed t(x, 1); ddm::launch_grid_post_from_pre(x->prec, x->kc, b, (int)k, x->seg_alist(m, j), x->seg_acount(m, j),
                                                      gpre(j), L.rec_items, x->at(L.grid_post), nullptr, st); }
      {
        Timed t(x, 4);
        if (x->kc.pcontact)
          ddm::launch_pcontact_adj(x->prec, x->kc, b, (int)L.nblk, (int)k, slot(j), gpost(j), adj[cur],
                                   x->at<double>(L.pose_bar), st);
        // one workgroup per tile: a persistent G2P adjoint ran slower (548 against 505 us per launch on the
        // 64-instance batch)
        ddm::launch_g2p_adj(x->prec, x->kc, b, tl, (int)L.nwg, slot(j), gpost(j), adj[cur], adj[1 - cur],
                            x->at(L.gvb), x->kc.det ? x->at(L.staging) : nullptr, st);
        if (x->kc.det) {
          // the staged windows, summed node by node in a fixed order
          ddm::launch_tile_slots(x->kc, tl, L.total_tiles, x->at<uint32_t>(L.tslot), st);
          ddm::launch_adj_windows(x->prec, x->kc, b, x->seg_alist(m, j), x->seg_acount(m, j), x->at(L.staging),
                                  x->at<const uint32_t>(L.tslot), x->at(L.gvb), st);
        }
      }
      if (treat) {
        Timed t(x, 9);
        treat_vectors(x, rec, TreatTarget{true, x->at(L.gvb), x->seg_alist(m, j), x->seg_acount(m, j), 3, false});
      }
      { Timed t(x, 5); ddm::launch_grid_adj(x->prec, x->kc, b, (int)k, x->seg_alist(m, j), x->seg_acount(m, j),
                                            gpre(j), L.rec_items, x->at(L.gvb), x->at(L.gb), x->at<double>(L.pose_bar), st); }
      if (treat) {
        Timed t(x, 9);
        treat_vectors(x, rec, TreatTarget{true, x->at(L.gb), x->seg_alist(m, j), x->seg_acount(m, j), 4, true});
      }
      { Timed t(x, 6); ddm::launch_p2g_adj(x->prec, x->kc, b, (int)L.nblk, slot(j), tau(j), x->at(L.gb),
                                           x->treat.mode == ddm::kTreatNone, adj[cur], adj[1 - cur],
                                           x->at<double>(L.pacc), st); }
      if (treat) {
        Timed t(x, 9);
        treat_vectors(x, rec, TreatTarget{false, adj[1 - cur]});
        if (rec) ddm::launch_treat_record(x->n_inst, acc, x->treat.mode != ddm::kTreatNone, x->stats_dev + stat_vals * k, st);
      }
      if (x->rec_sorted[(size_t)(s0 + j)]) {
        // the adjoint of a permutation is its inverse
        Timed t(x, 3);
        ddm::launch_unpermute(esz, adj[1 - cur], adj[cur], perm(j), L.rows, L.ntot, st);
      } else {
        cur = 1 - cur;
      }
    }
    const ddm_status s = launch_status();
    if (s != DDM_OK) return s;
  }
  ddm::launch_grad_final(x->kc, x->at<const ddm::InstDev>(L.inst), x->at<const double>(L.pacc),
                         x->at<const double>(L.pose_bar), x->at<const double>(L.pose_jac), (int)(k0 + n), dloss_dev,
                         grad_dev, st);
  // the replay re-binned segment states: the current state is binned afresh
  // before its next sub-step, and the last forward grid is gone
  x->need_sort = true;
  x->grid_valid = false;
  return launch_status();
}

namespace {

// The four calls of one optimiser pass, in order.
ddm_status run_pass(ddm_ctx* x, const void* x0, int32_t n_steps, const double* target, const double* dloss,
                    double* loss, double* grad) {
  ddm_status s = ddm_init_state(x, x0);
  if (s == DDM_OK) s = ddm_rollout(x, n_steps);
  if (s == DDM_OK) s = ddm_loss(x, target, loss);
  if (s == DDM_OK) s = ddm_backward(x, dloss, grad);
  return s;
}

void drop_graph(ddm_ctx* x) {
  if (x->gexec) (void)hipGraphExecDestroy(x->gexec);
  if (x->graph) (void)hipGraphDestroy(x->graph);
  x->gexec = nullptr;
  x->graph = nullptr;
}

}  // namespace

ddm_status ddm_set_grad_treatment(ddm_ctx* x, int32_t mode, double clip, double oom, double delta, double* stats_dev,
                                  int32_t stats_steps) {
  if (!x) return fail(DDM_EINVAL, "NULL context");
  if (mode < DDM_TREAT_NONE || mode > DDM_TREAT_NORM) return fail(DDM_EINVAL, "mode must be one of DDM_TREAT_*");
  if (mode == DDM_TREAT_CLIP && !(clip > 0)) return fail(DDM_EINVAL, "clip must be > 0");
  if (!std::isfinite(oom)) return fail(DDM_EINVAL, "oom must be finite");
  if (!(delta >= 0) || !std::isfinite(delta)) return fail(DDM_EINVAL, "delta must be finite and >= 0");
  if (stats_steps < 0 || (stats_steps > 0) != (stats_dev != nullptr))
    return fail(DDM_EINVAL, "stats_dev and stats_steps > 0 go together");
  if (mode == DDM_TREAT_NORM && x->cfg.deterministic)
    return fail(DDM_EINVAL, "normalisation reduces its 2-norm with atomics: not available in the deterministic mode");
  static_assert(DDM_TREAT_CLIP == ddm::kTreatClip && DDM_TREAT_SCALE == ddm::kTreatScale &&
                    DDM_TREAT_NORM == ddm::kTreatNorm, "treatment codes");
  x->treat = ddm::Treat{mode, clip, oom, delta};
  x->stats_dev = stats_dev;
  x->stats_steps = stats_steps;
  drop_graph(x);   // a captured pass holds the old setting
  return DDM_OK;
}

ddm_status ddm_pass(ddm_ctx* x, const void* x0_dev, int32_t n_steps, const double* target_hm_dev,
                    const double* dloss_dev, double* loss_dev, double* grad_dev, int32_t use_graph) {
  if (!x || !x0_dev || !target_hm_dev || !dloss_dev || !loss_dev || !grad_dev) return fail(DDM_EINVAL, "NULL argument");
  if (n_steps < 1 || n_steps > x->cfg.max_steps) return fail(DDM_EINVAL, "n_steps outside [1, max_steps]");
  if (!use_graph) return run_pass(x, x0_dev, n_steps, target_hm_dev, dloss_dev, loss_dev, grad_dev);
  const bool same = x->gexec && x->g_x0 == x0_dev && x->g_steps == n_steps && x->g_target == target_hm_dev &&
                    x->g_dloss == dloss_dev && x->g_loss == loss_dev && x->g_grad == grad_dev;
  if (!same) {
    drop_graph(x);
    // Capture: the sequence of kernels and copies is fixed by (n_steps, config),
    // and nothing in it waits for the host.  Timing events stay out of the graph.
    const int32_t timing = x->timing;
    x->timing = 0;
    DDM_HIP(hipStreamBeginCapture(x->stream, hipStreamCaptureModeThreadLocal));
    const ddm_status s = run_pass(x, x0_dev, n_steps, target_hm_dev, dloss_dev, loss_dev, grad_dev);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(x->stream, &g);
    x->timing = timing;
    if (s != DDM_OK) { if (g) (void)hipGraphDestroy(g); return s; }
    DDM_HIP(e);
    x->graph = g;
    const hipError_t ei = hipGraphInstantiate(&x->gexec, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) { drop_graph(x); return hip_check(ei, "instantiate the pass graph"); }
    x->g_x0 = x0_dev; x->g_steps = n_steps; x->g_target = target_hm_dev; x->g_dloss = dloss_dev;
    x->g_loss = loss_dev; x->g_grad = grad_dev;
    x->g_cur_off = x->cur_off; x->g_spare_off = x->spare_off;
    x->g_pid_off = x->pid_off; x->g_pid_spare_off = x->pid_spare_off;
  }
  DDM_HIP(hipGraphLaunch(x->gexec, x->stream));
  // host-side state after a pass (the capture set it the same way); the graph
  // ends with the state in the buffers that were current when it was captured
  x->cur_off = x->g_cur_off; x->spare_off = x->g_spare_off;
  x->pid_off = x->g_pid_off; x->pid_spare_off = x->g_pid_spare_off;
  x->steps = n_steps;
  x->initialised = true;
  x->recorded = true;
  x->rec_k0 = 0;
  x->rec_n = n_steps;
  x->loss_ready = true;
  x->need_sort = true;
  x->grid_valid = false;
  return DDM_OK;
}

ddm_status ddm_autotune(ddm_ctx* x, const char* cache_path, int32_t* sort_every_out) {
  Phase phase("ddm_autotune");
  if (!x) return fail(DDM_EINVAL, "NULL context");
  if (!x->initialised) return fail(DDM_ESTATE, "ddm_init_state first (the probe runs on the current state)");
  const Layout& L = x->L;
  int64_t n_part = 0;
  for (const auto& in : x->inst) n_part += in.n_particles;
  std::ostringstream key;
  key << "ddmpm dim=" << x->cfg.dim << " n_grid=" << x->cfg.n_grid << " prec=" << x->prec << " n_inst=" << x->n_inst
      << " particles=" << n_part << " ppc=" << x->cfg.ppc;
  int best = -1, best_w = 0;
  if (cache_path) {
    std::ifstream f(cache_path);
    std::string line;
    while (std::getline(f, line)) {
      const size_t k = line.find(" sort_every=");
      if (k == std::string::npos || line.compare(0, k, key.str()) != 0) continue;
      best = std::atoi(line.c_str() + k + 12);
      const size_t kw = line.find(" tile_workgroups=", k);
      best_w = kw == std::string::npos ? 0 : std::atoi(line.c_str() + kw + 17);
    }
  }
  if (best <= 0) {
    // Probe: the same forward sub-steps from the current state for every
    // candidate, the state restored before each.  The snapshot lives in
    // reverse-pass buffers (segment state 0, segment permutations), which hold
    // nothing between calls.  R first at the default workgroup count, then the
    // workgroup count at that R.
    const int P = std::min<int>(32, x->cfg.max_steps);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) cus = prop.multiProcessorCount;
    }
    void* snap = x->at(L.seg_state);
    void* pid_snap = x->at(L.seg_perm);
    x->rec_first = INT32_MAX;      // the snapshot overwrites recorded segments
    DDM_HIP(hipMemcpyAsync(snap, x->cur(), L.state_bytes, hipMemcpyDeviceToDevice, x->stream));
    DDM_HIP(hipMemcpyAsync(pid_snap, x->pid(), sizeof(uint32_t) * L.ntot, hipMemcpyDeviceToDevice, x->stream));
    const int saved_R = x->cfg.sort_every, saved_W = x->cfg.tile_workgroups;
    const int32_t saved_timing = x->timing;
    x->timing = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DDM_HIP(hipEventCreate(&e0));
    DDM_HIP(hipEventCreate(&e1));
    ddm_status st = DDM_OK;
    auto probe = [&](int R, int W, float* ms) -> ddm_status {
      DDM_HIP(hipMemcpyAsync(x->cur(), snap, L.state_bytes, hipMemcpyDeviceToDevice, x->stream));
      DDM_HIP(hipMemcpyAsync(x->pid(), pid_snap, sizeof(uint32_t) * L.ntot, hipMemcpyDeviceToDevice, x->stream));
      x->cfg.sort_every = R;
      x->cfg.tile_workgroups = W;
      x->need_sort = true;
      DDM_HIP(hipEventRecord(e0, x->stream));
      ddm_status r = DDM_OK;
      for (int i = 0; i < P && r == DDM_OK; ++i) {
        // pose rows 0 .. P-1: the cost of a sub-step does not depend on the pose
        if (sort_due(x, i)) {
          r = bin_current(x);
          x->need_sort = false;
        }
        if (r == DDM_OK) r = forward_step(x, i, x->tiles(), x->cur(), x->cur(), x->at(L.grid_pre), x->at(L.grid_post));
      }
      DDM_HIP(hipEventRecord(e1, x->stream));
      DDM_HIP(hipEventSynchronize(e1));
      DDM_HIP(hipEventElapsedTime(ms, e0, e1));
      return r;
    };
    const int cand_r[] = {2, 4, 8, 16, 32};
    float best_ms = 0.f;
    for (int rep = 0; rep < 2 && st == DDM_OK; ++rep) {          // the first round warms up
      for (int R : cand_r) {
        if (x->cfg.deterministic && R != cand_r[0]) continue;   // binned every sub-step: R has no effect
        float ms = 0.f;
        st = probe(R, 0, &ms);
        if (st == DDM_OK && rep == 1 && (best < 0 || ms < best_ms)) { best = R; best_ms = ms; }
      }
    }
    const int cand_w[] = {4 * cus, 8 * cus, 16 * cus, 32 * cus};
    best_w = 0;
    for (int W : cand_w) {
      if (st != DDM_OK || W >= L.nwg) break;       // at least one workgroup per tile already
      float ms = 0.f;
      st = probe(best, W, &ms);
      if (st == DDM_OK) st = probe(best, W, &ms);  // the second timing counts
      if (st == DDM_OK && ms < best_ms) { best_w = W; best_ms = ms; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    DDM_HIP(hipMemcpyAsync(x->cur(), snap, L.state_bytes, hipMemcpyDeviceToDevice, x->stream));
    DDM_HIP(hipMemcpyAsync(x->pid(), pid_snap, sizeof(uint32_t) * L.ntot, hipMemcpyDeviceToDevice, x->stream));
    DDM_HIP(hipStreamSynchronize(x->stream));
    x->timing = saved_timing;
    x->cfg.sort_every = saved_R;
    x->cfg.tile_workgroups = saved_W;
    if (st != DDM_OK) return st;
    if (cache_path) {
      std::ofstream f(cache_path, std::ios::app);
      if (f) f << key.str() << " sort_every=" << best << " tile_workgroups=" << best_w << "\n";
    }
  }
  x->cfg.sort_every = best;
  x->cfg.tile_workgroups = best_w;
  x->need_sort = true;            // the probe left the binning of another state
  x->grid_valid = false;
  if (sort_every_out) *sort_every_out = best;
  return DDM_OK;
}

ddm_status ddm_get_launch(const ddm_ctx* x, int32_t* sort_every, int32_t* tile_workgroups) {
  if (!x) return fail(DDM_EINVAL, "NULL context");
  if (sort_every) *sort_every = x->cfg.sort_every;
  if (tile_workgroups) *tile_workgroups = x->cfg.tile_workgroups;
  return DDM_OK;
}

ddm_status ddm_get_state(ddm_ctx* x, void* state_dev) {
  if (!x || !state_dev) return fail(DDM_EINVAL, "NULL argument");
  ddm::launch_export_state(x->kc, x->bufs(), (int)x->L.nblk, x->L.rows, x->L.esz, x->cur(), state_dev,
                           x->pid(), x->stream);
  return launch_status();
}

ddm_status ddm_set_state(ddm_ctx* x, const void* state_dev) {
  if (!x || !state_dev) return fail(DDM_EINVAL, "NULL argument");
  if (!x->initialised) return fail(DDM_ESTATE, "ddm_init_state first");
  DDM_HIP(hipMemcpyAsync(x->cur(), state_dev, x->L.state_bytes, hipMemcpyDeviceToDevice, x->stream));
  ddm::launch_reset_pid(x->bufs(), (int)x->L.nblk, x->pid(), x->stream);
  ddm::launch_fill_zero(x->at(x->L.gout), (int64_t)(x->L.grid_bytes / 4), 4, x->stream);
  x->grid_valid = false;
  x->recorded = false;
  x->loss_ready = false;
  x->need_sort = true;
  return launch_status();
}

ddm_status ddm_bin_keys(ddm_ctx* x, uint32_t* keys_dev, uint32_t* perm_dev) {
  if (!x || !keys_dev || !perm_dev) return fail(DDM_EINVAL, "NULL argument");
  if (!x->initialised) return fail(DDM_ESTATE, "ddm_init_state first");
  const Layout& L = x->L;
  uint32_t* keys[2] = {x->at<uint32_t>(L.keys0), x->at<uint32_t>(L.keys1)};
  uint32_t* vals[2] = {x->at<uint32_t>(L.vals0), x->at<uint32_t>(L.vals1)};
  ddm::launch_keys(x->prec, x->kc, x->bufs(), (int)L.nblk, x->cur(), keys[0], vals[0], x->stream);
  DDM_HIP(hipMemcpyAsync(keys_dev, keys[0], sizeof(uint32_t) * L.ntot, hipMemcpyDeviceToDevice, x->stream));
  const int r = ddm::radix_sort(keys, vals, L.ntot, L.max_key, x->at<uint32_t>(L.hist), x->at<uint32_t>(L.sums), x->stream);
  DDM_HIP(hipMemcpyAsync(perm_dev, vals[r], sizeof(uint32_t) * L.ntot, hipMemcpyDeviceToDevice, x->stream));
  return launch_status();
}

ddm_status ddm_get_grid(ddm_ctx* x, void* grid_dev) {
  if (!x || !grid_dev) return fail(DDM_EINVAL, "NULL argument");
  if (!x->grid_valid) return fail(DDM_ESTATE, "ddm_get_grid needs a forward sub-step since the last ddm_backward");
  ddm::launch_grid_export(x->prec, x->kc, x->at(x->L.grid_pre), x->at(x->L.grid_post), x->at<const uint32_t>(x->L.amask),
                          grid_dev, x->stream);
  return launch_status();
}

ddm_status ddm_eval_math(int32_t fn, const float* x_dev, float* y_dev, int64_t n, void* stream) {
  if (fn != 0 && fn != 1) return fail(DDM_EINVAL, "fn must be 0 (log1p) or 1 (expm1)");
  if (n < 0) return fail(DDM_EINVAL, "n < 0");
  if (n > 0 && (!x_dev || !y_dev)) return fail(DDM_EINVAL, "NULL argument");
  if (n > ((int64_t)1 << 40)) return fail(DDM_EINVAL, "n too large");
  ddm::launch_eval_math(fn, x_dev, y_dev, n, static_cast<hipStream_t>(stream));
  return launch_status();
}

ddm_status ddm_get_heightmap(ddm_ctx* x, double* hm_dev) {
  if (!x || !hm_dev) return fail(DDM_EINVAL, "NULL argument");
  const int npix = x->cfg.dim == 3 ? x->cfg.hm_res * x->cfg.hm_res : x->cfg.hm_res;
  DDM_HIP(hipMemcpyAsync(hm_dev, x->at(x->L.hm_val), sizeof(double) * (size_t)x->n_inst * npix, hipMemcpyDeviceToDevice,
                         x->stream));
  return DDM_OK;
}

ddm_status ddm_check(ddm_ctx* x, ddm_device_error* out) {
  if (!x) return fail(DDM_EINVAL, "NULL context");
  DDM_HIP(hipStreamSynchronize(x->stream));
  ddm::DevErr e;
  DDM_HIP(hipMemcpy(&e, x->at(x->L.err), sizeof(e), hipMemcpyDeviceToHost));
  if (out) {
    out->flags = e.flags;
    out->first_instance = e.first_inst;
    out->clamp_count = e.clamps;
  }
  if (e.flags & 1u) return fail(DDM_ENAN, "NaN or Inf in instance " + std::to_string(e.first_inst));
  if (e.flags & 2u) return fail(DDM_EDOMAIN, "a particle stencil left the grid in instance " + std::to_string(e.first_inst));
  if (e.flags & 16u)
    return fail(DDM_ENOMEM, "a recorded sub-step had more active grid blocks than grid_record_blocks (" +
                                std::to_string(x->cfg.grid_record_blocks) + "): the reverse pass is not valid");
  return DDM_OK;
}

ddm_status ddm_diagnostics(ddm_ctx* x, double* out_dev) {
  if (!x || !out_dev) return fail(DDM_EINVAL, "NULL argument");
  if (!x->initialised) return fail(DDM_ESTATE, "ddm_init_state first");
  static_assert(DDM_N_DIAG == 11, "diagnostics row");
  ddm::launch_diagnostics(x->prec, x->kc, x->bufs(), (int)x->L.nblk, x->cur(),
                          x->grid_valid ? x->at(x->L.grid_pre) : nullptr, x->active(), out_dev, x->stream);
  return launch_status();
}

int64_t ddm_steps_taken(const ddm_ctx* x) { return x ? x->steps : -1; }

int64_t ddm_instance_offset(const ddm_ctx* x, int32_t i) {
  if (!x || i < 0 || i >= x->n_inst) return -1;
  int64_t off = 0;
  for (int k = 0; k < i; ++k) off += pad_up(x->inst[k].n_particles, ddm::kBlock);
  return off;
}

ddm_status ddm_set_timing(ddm_ctx* x, int32_t groups) {
  if (!x) return fail(DDM_EINVAL, "NULL context");
  if (groups & ~DDM_TIMING_ALL) return fail(DDM_EINVAL, "timing groups outside DDM_TIMING_ALL");
  DDM_HIP(hipStreamSynchronize(x->stream));
  resolve_events(x);
  for (int g = 0; g < kTimingGroups; ++g) { x->t_ms[g] = 0.0; x->t_n[g] = 0; }
  x->timing = groups;
  return DDM_OK;
}

ddm_status ddm_read_timing(ddm_ctx* x, int32_t group, double* total_ms, int64_t* launches) {
  if (!x || group < 0 || group >= kTimingGroups) return fail(DDM_EINVAL, "bad context or group");
  DDM_HIP(hipStreamSynchronize(x->stream));
  resolve_events(x);
  if (total_ms) *total_ms = x->t_ms[group];
  if (launches) *launches = x->t_n[group];
  return DDM_OK;
}

void ddm_destroy(ddm_ctx* x) {
  if (!x) return;
  if (hipStreamSynchronize(x->stream) == hipSuccess) {
    drop_graph(x);
    for (const auto& e : x->events) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    for (hipEvent_t e : x->pool) (void)hipEventDestroy(e);
  }
  delete x;
}


// ---------------------------------------------------------------------------
// ddm_loss_noalloc: the loss of ddm_loss for one instance's positions, with
// every intermediate in one static device array (`scratch`) instead of a
// workspace.  Host code never names the array: its address on each device is
// taken once with hipGetSymbolAddress (that device current) and kept.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr size_t kNoAllocBytes = (size_t)8 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;     // per device: the address of `scratch` there

ddm_status scratch_address(void** out) {
  int dev = 0;
  DDM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[(size_t)dev]) {
    void* p = nullptr;
    DDM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[(size_t)dev] = p;
  }
  *out = g_scratch_ptr[(size_t)dev];
  return DDM_OK;
}

// Offsets of the pieces inside the static array for ntot particle slots and
// npix pixels (the largest case fits: checked at compile time below).
struct NoAllocLayout {
  size_t err, inst, poses, blk, pid, x, hm_bits, owner, dldh, hm_val, region, dldm, total;
};
constexpr NoAllocLayout noalloc_layout(int64_t ntot, int64_t npix, int dim, int esz) {
  NoAllocLayout L{};
  size_t off = 0;
  auto take = [&off](size_t bytes) { off = (off + 255) / 256 * 256; const size_t o = off; off += bytes; return o; };
  L.err = take(sizeof(ddm::DevErr));
  L.inst = take(sizeof(ddm::InstDev));
  L.poses = take((size_t)ddm::kPoseVals * esz);
  L.blk = take(sizeof(int) * (size_t)(ntot / ddm::kBlock));
  L.pid = take(sizeof(uint32_t) * (size_t)ntot);
  L.x = take((size_t)dim * ntot * esz);
  L.hm_bits = take(sizeof(unsigned long long) * (size_t)npix);
  L.owner = take(sizeof(unsigned int) * (size_t)npix);
  L.dldh = take(sizeof(double) * (size_t)npix);
  L.hm_val = take(sizeof(double) * (size_t)npix);
  L.region = take(sizeof(double));
  L.dldm = take(sizeof(double));
  L.total = take(0);
  return L;
}
static_assert(noalloc_layout(DDM_NOALLOC_MAX_PARTICLES, DDM_NOALLOC_MAX_PIXELS, 3, 8).total <= kNoAllocBytes,
              "the static scratch must hold the largest case");

}  // namespace

extern "C" {

ddm_status ddm_loss_noalloc(const ddm_config* cfg, const ddm_instance* inst, int32_t final_step, const void* x_dev,
                            const double* target_hm_dev, double* loss_dev, double* hm_dev, void* stream) {
  if (!cfg || !inst || !x_dev || !target_hm_dev || !loss_dev) return fail(DDM_EINVAL, "NULL argument");
  ddm_status s = validate(cfg, 1, inst);
  if (s != DDM_OK) return s;
  if (inst->n_particles > DDM_NOALLOC_MAX_PARTICLES)
    return fail(DDM_EINVAL, "n_particles above DDM_NOALLOC_MAX_PARTICLES (" +
                                std::to_string(DDM_NOALLOC_MAX_PARTICLES) + ")");
  const int64_t npix = cfg->dim == 3 ? (int64_t)cfg->hm_res * cfg->hm_res : cfg->hm_res;
  if (npix > DDM_NOALLOC_MAX_PIXELS)
    return fail(DDM_EINVAL, "hm_res^(dim-1) above DDM_NOALLOC_MAX_PIXELS (" + std::to_string(DDM_NOALLOC_MAX_PIXELS) + ")");
  if (cfg->w_emd != 0.0) return fail(DDM_EINVAL, "ddm_loss_noalloc has no EMD term: w_emd must be 0");
  if (final_step < -1 || final_step >= cfg->max_steps) return fail(DDM_EINVAL, "final_step outside [-1, max_steps)");
  void* base = nullptr;
  s = scratch_address(&base);
  if (s != DDM_OK) return s;
  char* sc = static_cast<char*>(base);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int prec = cfg->precision == DDM_F64 ? 1 : 0, esz = prec ? 8 : 4;
  const int64_t ntot = pad_up(inst->n_particles, ddm::kBlock), nblk = ntot / ddm::kBlock;
  const NoAllocLayout A = noalloc_layout(ntot, npix, cfg->dim, esz);
  // one instance, one pose row (that of final_step; the kernels read row 0)
  ddm_config c1 = *cfg;
  c1.max_steps = 1;
  ddm::KCfg kc = make_kcfg(c1, 1, ntot);
  const ddm::InstDev dev = make_instdev(*cfg, *inst, 0, 0, kc.nodes);
  double row[ddm::kPoseVals] = {0};
  if (final_step >= 0 && cfg->shovel) {
    ddm_config cp = *cfg;
    cp.max_steps = final_step + 1;
    std::vector<double> pose, jac;
    pose_table(cp, *inst, pose, jac);
    std::copy(pose.begin() + (size_t)final_step * 8, pose.begin() + (size_t)final_step * 8 + 8, row);
    row[8] = std::sin(row[3]);
    row[9] = std::cos(row[3]);
  }
  float rowf[ddm::kPoseVals];
  for (int k = 0; k < ddm::kPoseVals; ++k) rowf[k] = (float)row[k];
  ddm::launch_put_bytes(sc + A.inst, &dev, sizeof(dev), st);
  ddm::launch_put_bytes(sc + A.poses, prec ? (const void*)row : (const void*)rowf, (size_t)ddm::kPoseVals * esz, st);
  ddm::launch_fill_zero(sc + A.err, sizeof(ddm::DevErr) / 4, 4, st);
  ddm::launch_fill_zero(sc + A.blk, nblk, 4, st);            // every block belongs to instance 0
  ddm::Bufs b;
  b.inst = reinterpret_cast<const ddm::InstDev*>(sc + A.inst);
  b.blk_inst = reinterpret_cast<const int*>(sc + A.blk);
  b.poses = sc + A.poses;
  b.err = reinterpret_cast<ddm::DevErr*>(sc + A.err);
  uint32_t* pid = reinterpret_cast<uint32_t*>(sc + A.pid);
  ddm::launch_init_state(prec, kc, b, (int)nblk, x_dev, sc + A.x, pid, st, true);
  ddm::LossBufs lb;
  lb.hm_bits = reinterpret_cast<unsigned long long*>(sc + A.hm_bits);
  lb.owner = reinterpret_cast<unsigned int*>(sc + A.owner);
  lb.target = target_hm_dev;
  lb.hm_val = hm_dev ? hm_dev : reinterpret_cast<double*>(sc + A.hm_val);
  lb.dldh = reinterpret_cast<double*>(sc + A.dldh);
  lb.region = reinterpret_cast<double*>(sc + A.region);
  lb.dldm = reinterpret_cast<double*>(sc + A.dldm);
  lb.loss = loss_dev;
  ddm::launch_loss(prec, kc, b, (int)nblk, sc + A.x, pid, final_step >= 0 ? 0 : -1, lb, st);
  return launch_status();
}

}  // extern "C"
