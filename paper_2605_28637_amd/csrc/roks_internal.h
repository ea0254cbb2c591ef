// Internal declarations of the gfx950 ROKS library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/roks.h"

namespace roks {

// ---------------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------------
struct Error {
  roks_status code;
  std::string msg;
};

#define ROKS_HIP(call)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::roks::Error{ROKS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define ROKS_CHECK(cond, code, text)                             \
  do {                                                           \
    if (!(cond)) throw ::roks::Error{(code), std::string(text)}; \
  } while (0)

// ---------------------------------------------------------------------------
// plane-wave layout
// ---------------------------------------------------------------------------
// A "half column" is a line of stored plane waves with fixed (h, k): index 0
// is (0, 0) holding l >= 0; indices 1..nH are the columns with k > 0 or
// (k == 0, h > 0), each holding its whole l range [lmin, lmax].  Stored
// coefficients are ordered column by column, l ascending.  In the column
// buffers of the FFT the full sphere has ncol = 2 nH + 1 columns: column j
// (j <= nH) is half column j, column nH + j (j >= 1) its mirror (-h, -k).
struct ColDesc {
  int32_t h, k;       // Miller indices of the column (signed)
  int32_t base;       // storage index of (h, k, lmin)
  int32_t lmin, lmax; // stored l range
};

constexpr int kMaxShell = 4;  // closed, two open, virtual
constexpr int kMaxConf = 2;
constexpr int kMaxStages = 8;

struct FftPlan1D {
  int n = 0;
  int nstages = 0;
  int radix[kMaxStages] = {0};
};

FftPlan1D make_plan(int n);  // radices 8, 4, 2, 3, 5 (throws if n has other factors)

// the line-kernel split N = G P of a square plane (false: none built)
bool line_split(int n, int* G, int* P);
bool line_split_density(int n, int* G, int* P);

// ---------------------------------------------------------------------------
// the context
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Mlp;

constexpr int kDiisMaxHistory = ROKS_DIIS_MAX_HISTORY;

struct Ctx {
  // ---- problem description (host) ----
  double cell[3][3];
  double recip[3][3];
  double omega = 0;
  double ecut = 0;
  int N[3] = {0, 0, 0};
  int ntot = 0;
  int natoms = 0;
  std::vector<int32_t> spec_of;
  std::vector<double> pos;  // [natoms][3]
  struct Species {
    double A, sigma;
    std::vector<int32_t> l;
    std::vector<double> rp;
    std::vector<double> D;  // [nproj][nproj]
    std::vector<double> q;  // [nproj][nproj] overlap coefficients (zeros: S = 1)
  };
  std::vector<Species> species;
  int nb = 0;
  int nconf = 0;
  std::vector<uint8_t> occ;  // [nconf][2][nb]
  double cL[kMaxConf] = {0, 0};
  int xc = 0;
  int prec = 0;
  uint32_t flags = 0;

  // shells (groups of identical occupation patterns; order closed, open, virtual)
  int nshell = 0;
  int nsocc = 0;                                  // occupied shells (all but virtual)
  double shell_f[kMaxShell][kMaxConf][2] = {};    // f_X^{sigma L}
  double shell_w[kMaxShell] = {};                 // sum c_L f
  int shell_closed[kMaxShell] = {};
  int shell_virtual[kMaxShell] = {};
  std::vector<int32_t> band_shell;                // [nb]

  // plane waves
  int npw = 0;
  std::vector<int32_t> miller;  // [npw][3]
  std::vector<double> g2half;   // |G|^2 / 2
  int nH = 0, ncol = 0;
  std::vector<ColDesc> cols;    // nH + 1 half columns
  int hmax = 0;                 // max |h| over the sphere
  FftPlan1D plan[3];

  // projectors (atom-major, channel order of the species, l = 1 as x, y, z)
  int nproj = 0;
  std::vector<int32_t> proj_atom, proj_l, proj_m;
  std::vector<double> proj_rp;
  std::vector<int32_t> atom_proj_off, atom_proj_cnt;  // [natoms]
  std::vector<double> Dblk;       // per atom dense block, concatenated
  std::vector<int32_t> Dblk_off;  // [natoms]
  // overlap coefficients of S = 1 + sum q |beta><beta|, blocks laid out as
  // Dblk (same offsets); has_q: some q_kl != 0
  std::vector<double> Qblk;
  bool has_q = false;

  // ---- device ----
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // created on first use (side_stream): every stream a context holds takes a
  // share of the device's few hardware queues, idle or not
  // a second stream for the local force part beside the nonlocal part,
  // joined through events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int device = 0;
  std::vector<DevBuf> allocations;
  bool have_orbitals = false;
  bool potentials_valid = false;
  bool in_graph = false;  // launches being made for graph mode (one stream)
  // the vectors whose z pass (G -> r) d_T holds, in tier T_prec (nullptr:
  // none); an energy evaluation sets it, every other writer of d_T clears it
  const void* T_src = nullptr;
  int T_prec = -1;
  const double* zskip = nullptr;  // graph mode: the apply's z pass skip flag

  // device arrays (FP64 tier; FP32 copies live in the *_f32 members)
  int32_t* d_miller = nullptr;
  double* d_g2 = nullptr;        // |G|^2/2
  ColDesc* d_cols = nullptr;
  int32_t* d_colpos = nullptr;   // [ncol][2] (h mod N1, k mod N2)
  double2* d_tw[3] = {nullptr, nullptr, nullptr};  // exp(-2 pi i k / N_d)
  float2* d_tw32[3] = {nullptr, nullptr, nullptr};
  float* d_vsh32 = nullptr;      // FP32 tier copies of the shell and channel potentials
  float* d_vloc32 = nullptr;
  double* d_vext = nullptr;      // [N3][N1][N2]
  double2* d_B = nullptr;        // [nproj][npw]
  // BF16x3 tier: the projector table split into hi / lo BF16 rows of a
  // multiple of 64, projector-major [2][nproj][Kp] and coefficient-major
  // [2][2 npw][npp], and the band-side split buffer [2][nb][max(Kp, npp)]
  bool bf3 = false;
  bool bsplit_valid = false;
  uint16_t* d_bsplit = nullptr;
  uint16_t* d_bsplit_t = nullptr;
  uint16_t* d_xsplit = nullptr;
  uint16_t* d_fsplit = nullptr;   // force field operands [2][nproj + 2 npw][nbp]
  int32_t* d_proj_atom = nullptr;
  double* d_Dblk = nullptr;
  int32_t* d_Dblk_off = nullptr;
  double* d_Qblk = nullptr;      // with has_q
  double2* d_Spsi = nullptr;     // with has_q: [nb][npw] S|psi_n> of the last gradient
  int32_t* d_atom_proj_off = nullptr;
  int32_t* d_atom_proj_cnt = nullptr;
  int32_t* d_band_shell = nullptr;

  double2* d_psi = nullptr;      // [nb][npw] current orbitals
  double2* d_in = nullptr;       // [nb][npw] staging for caller vectors
  double2* d_Y = nullptr;        // [nb][npw]
  double2* d_gI = nullptr;
  double2* d_p = nullptr;
  double2* d_S = nullptr;
  double2* d_Sold = nullptr;
  double2* d_Pt = nullptr;       // trial vectors
  double2* d_trial[2] = {nullptr, nullptr};  // trial orbitals (an accepted one swaps with d_psi)
  double2* d_w1 = nullptr;       // scratch band array, followed by d_Sold
  double* d_m12 = nullptr;       // [nb][2 nb]: <psi|w1> and <psi|S_old> side by side
  double2* d_T = nullptr;        // [npairs][N3][ncol] column buffer
  double* d_rho_part = nullptr;  // [nchunk][nsocc][ntot]
  double* d_rho = nullptr;       // [nsocc][ntot]
  double* d_vloc = nullptr;      // [nconf][2][ntot]
  double* d_vsh = nullptr;       // [nsocc][ntot]
  // hybrid exact exchange (exx.hip): real-space orbitals [nb][ntot] of the
  // last potentials' orbitals, 3 complex work grids, pair integrals,
  // reduction partials, the weights W[X][m] = sum_L c_L sum_s f_X f_m, and
  // E_x^HF per configuration (host)
  double exx = 0.0;
  double* d_exx_u = nullptr;
  double2* d_exx_g = nullptr;
  double* d_exx_I = nullptr;
  double* d_exx_part = nullptr;
  double* d_exx_W = nullptr;
  double exx_E[kMaxConf] = {0.0, 0.0};
  double2* d_gga = nullptr;      // PBE: [4][ntot] packed spin fields (spectra, gradients)
  double* d_gga_e = nullptr;     // PBE: [nconf][ntot] energy densities
  double2* d_fft = nullptr;      // [ntot]
  double* d_P = nullptr;         // [nproj][nb]
  double* d_DP = nullptr;        // [nproj][nb]
  double* d_part = nullptr;      // reduction partials
  double* d_red = nullptr;       // reduced scalars
  double* d_gemm_part = nullptr;  // split-K partials
  double* d_Qpart = nullptr;     // [npairs][N3][2][nsocc]
  double* d_Q = nullptr;         // [nb][nsocc]
  double* d_kin = nullptr;       // [nb]
  double* d_enl = nullptr;       // [nb]
  double* d_bandv = nullptr;     // [8][nb] per-band scratch scalars
  double* d_cg = nullptr;        // [8 + nb]: [0] A-part of <p|g>, [1] beta, [8 + n] <p_n|g_n>
  // nb x nb matrices
  double *d_theta = nullptr, *d_R = nullptr, *d_kappa = nullptr, *d_A = nullptr, *d_D = nullptr,
         *d_Dold = nullptr, *d_gram = nullptr, *d_Linv = nullptr, *d_U = nullptr,
         *d_M = nullptr, *d_m1 = nullptr, *d_m2 = nullptr, *d_m3 = nullptr, *d_Mkeep = nullptr,
         *d_Ukeep = nullptr;
  double* d_SS = nullptr;        // <S_m|S_n> of the current search direction
  double* d_ex = nullptr;        // [5][nb][nb] scratch of the multi-kernel exponential (nb > 78)
  double* d_PSold = nullptr;     // <psi|S_old> left by the last commit
  int psold_iter = -1;           // the iteration it belongs to (-1: none)
  double* d_P0 = nullptr;        // [nproj][nb] <beta|psi> at the start of the line search
  double* d_PS = nullptr;        // [nproj][nb] <beta|S>
  int32_t* d_flag = nullptr;     // device status flags
  double* d_force = nullptr;     // [natoms][3]
  double* d_force_loc = nullptr; // [natoms][3] local part (side stream)
  double* d_gcart = nullptr;     // [3][npw] Cartesian G of the stored coefficients (forces)
  double* d_phi = nullptr;       // [nproj][npw] force field sum_n w_n (D P)_in psi_n, then 3 nproj sums
  void* d_atoms = nullptr;       // per-atom position and local-well parameters
  void* d_projinfo = nullptr;    // per-projector atom, l, m, radius
  double* d_dP = nullptr;        // [nproj][nb] derivative projections
  double2* d_hch = nullptr;      // [4][nb][npw] multi-channel apply output (lazy)
  double* d_scal = nullptr;      // [16 + 2 nb]: reduced energy sums, then kin, enl
  // pinned, coherent host mirrors written by the kernels (read after a
  // synchronisation)
  double* h_scal = nullptr;      // [16 + 2 nb]: mirror of d_scal
  double* h_stage = nullptr;     // [kStage + 4 nb]
  int32_t* h_flag = nullptr;     // [16]
  double* h_force = nullptr;     // [natoms][3] forces (nonlocal kernel writes them)
  double* hd_scal = nullptr;     // device view of h_scal
  double* hd_stage = nullptr;    // device view of h_stage (kernels write it directly)
  bool normD_pending = false;    // ||D||_1 queued into h_stage, not yet synchronised
  int32_t* hd_flag = nullptr;    // device view of h_flag
  double* hd_force = nullptr;    // device view of h_force
  double* d_m4 = nullptr;
  double* d_kinw_shell = nullptr;  // [nb] shell weight of each band (0 for virtual)
  double* d_ones = nullptr;        // [nb] ones
  int32_t* d_potidx = nullptr;     // [6][nb]: shell potential per band, channel 0..3, closed shell
  double* d_kinw_closed = nullptr; // [nb] weight of the closed shell (F^c for every band)

  int npairs = 0;
  int nchunk = 0;
  // the device's static scratch of the allocation-free apply (its address on
  // this context's device) and whether a call runs on it (no autotuning then)
  void* d_noalloc = nullptr;
  bool no_alloc = false;
  // plane passes with the lines in registers (square planes N = G P): G and
  // P (0: not available, the LDS-plane kernels run), per-column LDS index and
  // per-row k range of the pruned [2 hmax + 1][N + 1] plane
  int lines_G = 0, lines_P = 0;
  int dlines_G = 0, dlines_P = 0;  // the split of the density passes
  int32_t* d_colidx = nullptr;   // [ncol]
  int32_t* d_krange = nullptr;   // [2 hmax + 1][2] signed k range of each row
  size_t part_capacity = 0;      // doubles in d_part
  size_t gemm_part_capacity = 0;

  // ---- CG state (host mirrors of scalars) ----
  bool have_old = false;
  double pg_old = 0;
  double dt = 0.5;
  int iteration = 0;

  // ---- graph mode (graph.hip): CG iterations decided on the device ----
  double* d_gstate = nullptr;      // state block and per-band scratch
  double* d_gfocc = nullptr;       // [nconf][nb] occupation of each band
  // the first trial's potentials and projections (kept for the next
  // iteration when that trial is taken)
  double* d_gvsh = nullptr;
  double* d_gvloc = nullptr;
  float* d_gvsh32 = nullptr;
  float* d_gvloc32 = nullptr;
  double* d_gP = nullptr;
  double* d_gscal = nullptr;       // reduced sums, as d_scal
  double* d_gPSt = nullptr;        // t <beta|S> of a trial
  double* h_gmirror = nullptr;     // pinned copy of the state block
  double* hd_gmirror = nullptr;    // its device view
  double* h_grec = nullptr;        // pinned per-iteration records
  double* hd_grec = nullptr;
  int grec_cap = 0;                // iterations the records hold
  hipGraphExec_t graph_exec = nullptr;  // the captured iterations
  int graph_k = 0;                 // how many (0: none captured)
  int graph_prec = 0;              // the tier and flags it was captured with
  uint32_t graph_flags = 0;
  const Mlp* graph_mlp = nullptr;  // and the network attached
  // the buffers the capture baked in (orbitals, trials, projections, which
  // the host CG trades by pointer)
  void* graph_bufs[5] = {};

  // ---- cached results of the last energy evaluation ----
  roks_energies last_e{};
  std::string last_error;

  // periodic CG restart (0: never) and the steps since the last one
  int restart_period = 0;
  int since_restart = 0;
  // DIIS (diis.hip): kept iterates [slot][psi, e][nb][npw] for up to
  // kDiisMaxHistory slots, per-band dots [1 + history][nb], B over slots,
  // the kept slots oldest first
  double2* d_diis = nullptr;
  double* d_diis_dots = nullptr;
  std::vector<double> diis_B;
  std::vector<int> diis_order;
  int diis_hist = 0;
  bool diis_asym = false;

  // ---- learned preconditioner ----
  Mlp* mlp = nullptr;               // attached network (not owned)
  int nsh = 0;                      // distinct |G|^2 values ("G shells")
  std::vector<double> g2sh;         // their |G|^2/2
  std::vector<int32_t> gshell;      // shell of every stored G
  std::vector<int32_t> sh_perm, sh_off;  // G sorted by shell, shell offsets
  int32_t* d_gshell = nullptr;
  int32_t* d_sh_perm = nullptr;
  int32_t* d_sh_off = nullptr;
  double* d_g2sh = nullptr;
  float* d_feat = nullptr;          // [nb][nsh][3]
  float* d_scale = nullptr;         // [nb][nsh]
  int32_t* d_valid = nullptr;       // [nb]: band has a nonzero g_I
  // recording of (psi_i, plain Teter K g_I, features) for training
  int rec_max = 0, rec_stride = 1, rec_count = 0;
  double2* d_rec_psi = nullptr;     // [rec_max][nb][npw]
  double2* d_rec_kg = nullptr;
  float* d_rec_feat = nullptr;      // [rec_max][nb][nsh][3]
  int32_t* d_rec_valid = nullptr;   // [rec_max][nb]
  double* d_rec_ekin = nullptr;     // [rec_max][nb] <n|T|n> of the iterate
  int32_t* d_rec_sel = nullptr;     // [nb] selected bands during collection
  double* d_mom = nullptr;          // [3][nb][nsh] moments scratch

  // ---- diagnostics: per-kernel event pairs on `stream` ----
  bool timing = false;
  std::string timing_only;  // record only this kernel family (empty: all)
  struct Timed {
    std::string name;
    hipEvent_t a, b;
    double bytes, flops;  // algorithmic HBM bytes and flops of the launch
  };
  std::vector<Timed> timed;
};

// ---------------------------------------------------------------------------
// learned rescaling of the Teter preconditioner (mlp.hip)
// ---------------------------------------------------------------------------
constexpr int kMlpWidth = 64;
constexpr int kMlpFeat = 3;
constexpr int kMlpParams = kMlpWidth * kMlpFeat + kMlpWidth + kMlpWidth * kMlpWidth + kMlpWidth +
                           kMlpWidth + 1;  // 4481

struct Mlp {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<DevBuf> allocations;
  float* d_p = nullptr;      // FP32 master parameters
  uint16_t* d_pb = nullptr;  // BF16 copy read by every evaluation
  float *d_m = nullptr, *d_v = nullptr, *d_g = nullptr;  // Adam moments, gradient
  int adam_t = 0;
  double* d_loss = nullptr;  // [2]: mean loss, counted bands
  // training set: one sample per (band, G shell), grouped by recorded
  // iterate (segments)
  int S = 0, Scap = 0, nseg = 0;
  size_t seg_cap = 0;
  std::vector<int32_t> band_off{0};  // segment offsets (host copy), nseg + 1
  float* d_X = nullptr;              // [Scap][3]
  double* d_abg = nullptr;           // [3][Scap]: alpha, beta, gamma
  int32_t* d_band_of = nullptr;      // [Scap] segment of every sample
  int32_t* d_band_off = nullptr;     // [nseg + 1]
  // scratch sized with the training set
  float *d_o = nullptr, *d_do = nullptr;
  float *d_H1 = nullptr, *d_DZ2 = nullptr, *d_DZ1 = nullptr, *d_HD3 = nullptr;  // [64][Scap]
  double* d_ABC = nullptr;  // [nseg][3]
  double* d_Lseg = nullptr;
  int32_t* d_ok = nullptr;
  float* d_part = nullptr;  // gradient partials [chunks][params]
  size_t part_cap = 0;
  std::string last_error;
};

// Records HIP events around the launches in its scope when timing is on,
// with the launch's algorithmic byte and flop counts.
struct KernelTimer {
  Ctx& c;
  int idx = -1;
  KernelTimer(Ctx& ctx, const char* name, double bytes = 0.0, double flops = 0.0);
  ~KernelTimer();
};

// host setup (setup.cpp)
void grid_rule(const double cell[3][3], double ecut, int grid[3]);
void build_problem(Ctx& c, const roks_system* sys);
void build_sphere(Ctx& c);
void build_projectors(Ctx& c);

// device setup and memory (device.cpp)
void init_device(Ctx& c, void* stream);
void free_device(Ctx& c);
// the side stream and its fork/join events, created on first use
void ensure_side_stream(Ctx& c);
void clear_timing(Ctx& c);
void upload_static(Ctx& c);   // sphere tables, twiddles, V_ext, projectors
void upload_positions(Ctx& c);

// kernels launchers -----------------------------------------------------------
// fft.hip
// The column buffer T and the potential grids are in the context's tier
// (double for ROKS_FP64, float for ROKS_FP32); band vectors are FP64.
// skip (device, nullable): when *skip != 0 the launch does nothing (graph
// mode: the buffer already holds the transform)
void launch_zpass_bwd(Ctx& c, const double2* vecs, int nvec, void* T, int npairs,
                      const double* skip = nullptr);
// pot holds npot (1..3) grids; potidx[n] selects band n's grid (-1: zero);
// nQ > 0 also accumulates <n|V^X|n> for the first nQ grids into Qpart
void launch_plane_apply(Ctx& c, void* T, int npairs, const void* pot, int npot,
                        const int32_t* potidx, int nvec, double* Qpart, int nQ);
// whether the FP32 tier runs the density planes in FP32 (else FP64)
bool fp32_density_planes(const Ctx& c);
void launch_plane_density(Ctx& c, const void* T, int npairs, double* rho_part, int nchunk);
void launch_zpass_fwd(Ctx& c, const void* T, int npairs, const double2* vecs, int nvec,
                      const double* kinw, double2* Y);
void launch_fft3d(Ctx& c, double2* data, int sign);  // FP64 full-grid transform
// V_H(G) = 4 pi rho(G) / (G^2 N^3) (0 at G = 0) of a packed grid, in place:
// the forward transform, the multiply and the inverse transform
void launch_hartree_fft(Ctx& c, double2* data);

// fields.hip
void launch_vext(Ctx& c);
void launch_projectors(Ctx& c, double2* B, int deriv_axis);
// shell densities from the chunk partials, and the packed configuration
// densities in d_fft for the Hartree step that follows
void launch_density_reduce(Ctx& c, const double* rho_part, int nchunk, double* rho);
// V_H per configuration from the packed densities in d_fft
void launch_hartree(Ctx& c);
// hybrid exact exchange (exx.hip).  exx_orbitals: the real-space orbitals
// of orb (kept for the applies of the same orbitals); exx_energies: E_x^HF
// per configuration into exx_E (synchronises); exx_apply: out[n] += a
// sum_m rowW[n][m] psi_m V[psi_m v_n] for the nvec rows of vecs (rowW host
// [nvec][nb], the minus sign of K included), with Iout the pair integrals
// I[n][m] kept for exx_shell_expectations, which adds a <n|K^X|n> to d_Q
void exx_orbitals(Ctx& c, const double2* orb);
void exx_energies(Ctx& c);
void exx_apply(Ctx& c, const double2* vecs, int nvec, const double* rowW, double2* out, double* Iout);
void exx_shell_expectations(Ctx& c);
// PBE (ROKS_XC_PBE): write = true forms V_loc, the shell potentials and the
// energy partial sums (after launch_hartree), false the energy sums only
void launch_gga(Ctx& c, double* part, int nblocks, bool write);
void launch_xc_potentials(Ctx& c, double* part, int nblocks);
int xc_blocks(const Ctx& c);
void launch_band_kinetic(Ctx& c, const double2* vecs, int nvec, double* out);
void launch_nl_energy(Ctx& c, const double* P, double* out, double* mirror = nullptr);
void launch_apply_D(Ctx& c, const double* P, const double* w, double* DP);
// QP[i][n] = sum_j q_ij P[j][n] over the atom's projectors (has_q)
void launch_apply_Q(Ctx& c, const double* P, double* QP);
// G[m][n] = (theta_mn + theta_nm) / 2 for occupied m and n, else 0
void launch_overlap_multipliers(Ctx& c, const double* theta, double* G);
// energy-only evaluation: xc and external sums without potentials, and the
// Hartree integrals from the forward transform (partials [block][2])
void launch_xc_energy(Ctx& c, double* part, int nblocks);
void launch_hartree_energy(Ctx& c, double* part, int nblocks);
// column sums of part [nrows][ncols] into out (and mirror); with part2, its
// ncols2 columns ([nrows][ncols2]) follow in out in the same launch
void launch_reduce_columns(Ctx& c, const double* part, int nrows, int ncols, double* out,
                           double* mirror = nullptr, const double* part2 = nullptr,
                           int ncols2 = 0);
void launch_to_float(Ctx& c, const double* in, float* out, size_t n);
void launch_reduce_strided(Ctx& c, const double* part, int nouter, int ninner, int ncols,
                           double scale, double* out);
void launch_local_force(Ctx& c, const double2* rhoG, double* out_part, int nblk);
void launch_pack_rho_weighted(Ctx& c);
size_t atom_info_bytes();
size_t proj_info_bytes();
// forces: out = -(loc + nonlocal part) from the force field phi [nproj][npw]
// (Phi_i = sum_n w_n (D P)_in psi_n); part: 3 nproj doubles of scratch
void launch_nl_force(Ctx& c, const double* phi, double* part, const double* loc, double* out);
// the Cartesian components of every stored G, [3][npw]
void launch_gcart(Ctx& c, double* gcart);

// tile_gemm.hip: C = alpha op(A) op(B) + beta Cin on the FP64 matrix cores,
// 128 x 128 tiles staged in LDS, split-K over ks chunks (ks <= 0: chosen
// from the shape) summed in chunk order.  alay 0: op(A)[m][k] = A[m lda + k],
// 1: A[k lda + m]; blay 0: op(B)[k][n] = B[n ldb + k], 1: B[k ldb + n];
// B2 (blay 1, nullable): op(B) + b2 op(B2); half_weights (alay = blay = 0):
// the Gamma weight of k (1 for k < 2, else 2); Cin nullable (C)
void tile_gemm(Ctx& c, int M, int N, int K, const double* A, int lda, int alay, const double* B,
               int ldb, int blay, const double* B2, double b2, double* C, int ldc, const double* Cin,
               int ldcin, double alpha, double beta, bool half_weights, int ks);
int tile_gemm_splits(const Ctx& c, int M, int N, int K);
// C = alpha (sum of the ks split-K chunks in d_gemm_part, each M x N) +
// beta Cin, the chunks added in order
void launch_tile_reduce(Ctx& c, int ks, int M, int N, double* C, int ldc, const double* Cin, int ldcin,
                        double alpha, double beta);

// bf16x3.hip: the products with the projector table, in FP64 or, with the
// BF16x3 tier on (c.bf3), on the BF16 matrix cores over split operands.
// nrows <= nb rows of X (length 2 npw, leading dimension ldx):
// C[p][n] = <beta_p|x_n> (stored-half weights)
void proj_wdot(Ctx& c, int nrows, const double* X, int ldx, double* C, int ldc);
// the force field Phi[p] = sum_n DPw[p][n] x_n (all nb bands of X; DPw
// nproj x nb, leading dimension lddp), [nproj][2 npw]
void proj_field(Ctx& c, const double* DPw, int lddp, const double* X, int ldx, double* Phi);
// Y[n] += sum_p DP[p][n] beta_p (DP nproj x nrows, leading dimension lddp)
void proj_expand(Ctx& c, int nrows, const double* DP, int lddp, double* Y, int ldy);

// linalg.hip
void gemm_wdot(Ctx& c, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
               double* C, int ldc, double alpha, double beta, bool half_weights);
void gemm_expand(Ctx& c, int N, int K, int Mdim, const double* M, int ldm, bool transM,
                 const double* X, int ldx, double* Y, int ldy, double alpha, double beta);
// the same with the beta term read from Yin (Y = alpha M^T X + beta Yin;
// Yin may be Y): saves a copy when the result goes to another buffer
void gemm_expand_to(Ctx& c, int N, int K, int Md, const double* M, int ldm, bool transM,
                    const double* X, int ldx, const double* Yin, int ldyin, double* Y, int ldy,
                    double alpha, double beta);
// Y = alpha M^T (X + dX2 X2) + beta Yin, X2 (same layout as X) added while
// loading
void gemm_expand_sum(Ctx& c, int N, int K, int Md, const double* M, int ldm, bool transM,
                     const double* X, const double* X2, double dX2, int ldx, const double* Yin,
                     int ldyin, double* Y, int ldy, double alpha, double beta);
// C = alpha op(A) op(B) + beta C + diag I
void gemm_small(Ctx& c, int M, int N, int K, const double* A, int lda, bool tA, const double* B,
                int ldb, bool tB, double* C, int ldc, double alpha, double beta, double diag = 0.0);
// the same with op(A + a2 A2) (A2 of A's layout, may be null)
void gemm_small2(Ctx& c, int M, int N, int K, const double* A, const double* A2, double a2, int lda,
                 bool tA, const double* B, int ldb, bool tB, double* C, int ldc, double alpha,
                 double beta, double diag);
void band_dots(Ctx& c, const double2* X, const double2* Y, int nvec, int mode, double* out);
// both weightings in one pass: out0 plain, out1 |G|^2/2 (either may be null)
void band_dots2(Ctx& c, const double2* X, const double2* Y, int nvec, double* out0, double* out1,
                double* mirror0 = nullptr, double* mirror1 = nullptr);
void axpby(Ctx& c, size_t n, double a, const double* x, double b, const double* y, double* out);
void cholesky_inverse(Ctx& c, const double* G, int n, double* Linv, int32_t* flag);
void set_identity(Ctx& c, double* A, int n, double diag);
// the truncated exponential series of X (n x n) to degree m by the
// Paterson-Stockmeyer scheme (blocks of three) in taylor_products(m) matrix
// products; X2, X3, w0, w1 scratch, the result in w0 or w1 (returned)
int taylor_products(int m);
double* taylor_ps(Ctx& c, int n, int m, const double* X, double* X2, double* X3, double* w0, double* w1);
// out = a in + d I (n x n)
void scale_shift(Ctx& c, const double* in, int n, double a, double d, double* out);
void matrix_norm1(Ctx& c, const double* A, int n, double* out);
// open_out: also the open-shell coupling (two open shells only)
void launch_subspace(Ctx& c, double* open_out = nullptr);
// the virtual block of R from <m|F^c|n> already in R[v0.., v0..] (upper
// triangle mirrored; with canonicalisation kappa and the Jacobi angles)
void launch_virtual_block(Ctx& c, int v0);
bool expm_in_lds(const Ctx& c);
// raise a kernel's dynamic LDS limit to bytes (a runtime call only the first
// time a larger size is asked for on the current device)
void allow_dynamic_lds(const void* kernel, size_t bytes);
// Cholesky inverse of G and U = exp(delta D) in one launch of two workgroups
// (nb within the single-workgroup limits of both)
void launch_chol_expm_lds(Ctx& c, const double* G, double ga, double gd, double* Linv, int32_t* flag,
                          const double* D, double delta, double* U);
void launch_expm_lds(Ctx& c, const double* D, double delta, double* U, hipStream_t stream);
void launch_asym_dot(Ctx& c, const double* A, const double* theta, double* out,
                     double* mirror = nullptr);
// out0[n] = <X_n|Y_n> (and mirror0[n]) for n < nvec, and aout = sum A (theta -
// theta^T) (and amirror), in one launch
void band_dots_asym(Ctx& c, const double2* X, const double2* Y, int nvec, double* out0,
                    double* mirror0, const double* A, const double* theta, double* aout,
                    double* amirror);
// S = p + beta w (n1 values), D = A + beta D_old (n2 values) with beta =
// (sum_n pgb[n] + asym[0] / 2) / pg_old formed on the device (kept in beta_out)
void cg_directions_dev(Ctx& c, size_t n1, const double* p, const double* w, double* S, size_t n2,
                       const double* A, const double* Dold, double* D, const double* asym,
                       const double* pgb, double pg_old, double* beta_out);
void launch_teter(Ctx& c, const double* gTg, const double* gg, const double2* g, const double* bandw,
                  double2* out);

// mlp.hip
void mlp_init(Mlp& m, const float* theta, uint64_t seed);  // theta NULL: seeded init
void mlp_free(Mlp& m);
void mlp_set_params(Mlp& m, const float* host);
void mlp_forward(Mlp& m, const float* dX, int S, float* d_o, float* d_s, hipStream_t stream);
void mlp_loss_grad(Mlp& m, double* d_out);  // loss (and count) into d_out, gradient into d_g
void mlp_adam(Mlp& m, double lr);
void mlp_clear_samples(Mlp& m);
void build_gshells(Ctx& c);
void launch_features(Ctx& c, const double* gTg, const double* gg, const double* ekin);
void launch_teter_scaled(Ctx& c, const double* gTg, const double* gg, const double2* g,
                         const double* bandw, double2* out);
void record_iterate(Ctx& c, const double* gTg, const double* gg, const double* ekin);
void polar_factor(Ctx& c, double* X, int n, double* T, double* Xn, bool* converged);
void collect_records(Ctx& c, Mlp& m, int* used, int* skipped);

// solver (solver.cpp)
void compute_potentials(Ctx& c, const double2* orbitals, roks_energies* e);
// every launch of it, no synchronisation (energies reduced into d_scal and
// its pinned mirror); have_P: the projections of orb are already in d_P
void compute_potentials_async(Ctx& c, const double2* orb, bool have_P, bool energy_only);
void ensure_potentials(Ctx& c);
void apply_operator(Ctx& c, const double2* vecs, uint32_t mask, double2* out, bool want_Q);
// want_vv: also the virtual-virtual block of R, <m|F^c|n> (always with
// ROKS_FLAG_CANONICALIZE, whose Jacobi angles rotate that block)
void energy_gradient(Ctx& c, roks_energies* e, double* open_out = nullptr, bool want_vv = false);
void pcg_step(Ctx& c, roks_step_info* info);
// stream-ordered helpers of the host-side solvers
inline void to_host(Ctx& c, void* dst, const void* src, size_t bytes) {
  ROKS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c.stream));
  ROKS_HIP(hipStreamSynchronize(c.stream));
}
inline void sync(Ctx& c) { ROKS_HIP(hipStreamSynchronize(c.stream)); }
inline void copy_dev(Ctx& c, void* dst, const void* src, size_t bytes) {
  ROKS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c.stream));
}
inline double* dbl(double2* p) { return reinterpret_cast<double*>(p); }
inline const double* dbl(const double2* p) { return reinterpret_cast<const double*>(p); }

// DIIS on the residual of Eq. residual_frank (diis.hip); reset_diis drops
// the kept iterates
void diis_step(Ctx& c, const roks_diis_params& p, roks_diis_info* info);
void reset_diis(Ctx& c);
// S|psi_n> of the current orbitals as left by the last energy_gradient
// (d_Spsi with overlap coefficients, else the orbitals themselves)
const double2* overlap_psi(const Ctx& c);
void orthonormalize(Ctx& c, double2* vecs);
// the allocation-free operator application (noalloc.hip): its scratch is a
// file-scope device array of this size on every device
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
void init_noalloc_scratch(Ctx& c);
// roks_apply_h_d's work with the scratch in that array (vecs NULL: the
// orbitals); the potentials must be current
void apply_noalloc(Ctx& c, const double2* vecs, uint32_t mask, double2* out);
// the smallest trial step the next line search can take (its halvings of the
// current trial step)
double smallest_trial_step(const Ctx& c);
// Im c_n(0) = 0 for nvec bands (real orbitals)
void launch_zero_g0_imag(Ctx& c, double2* vecs, int nvec);
void forces(Ctx& c, double* f_host);
void reset_cg(Ctx& c);
// graph mode (graph.hip): k device-decided CG iterations replayed from one
// captured graph; returns the leading accepted ones (info: k records)
int graph_steps(Ctx& c, int k, roks_step_info* info);
bool graph_eligible(const Ctx& c);  // within graph mode's scope
void free_graph(Ctx& c);       // the captured graph
void free_graph_mode(Ctx& c);  // and the pinned records

// helpers
template <typename T>
T* dalloc(Ctx& c, size_t count) {
  void* p = nullptr;
  size_t bytes = count * sizeof(T);
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) throw Error{ROKS_ERR_OOM, "hipMalloc failed"};
  ROKS_HIP(hipMemsetAsync(p, 0, bytes, c.stream));
  c.allocations.push_back({p, bytes});
  return static_cast<T*>(p);
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// the CG trial step: its bounds, its first value and the halvings of one
// line search
constexpr double kDtMin = 0.1, kDtMax = 2.0, kDtInit = 0.5;
constexpr int kHalvings = 4;

constexpr int kStage = 16;  // scalar slots ahead of the per-band ones in h_stage
constexpr int kStageNormD = 3;  // h_stage slot of ||D||_1 for the line search

}  // namespace roks

// the opaque handle of the C ABI
struct roks_ctx_s {
  roks::Ctx c;
};
