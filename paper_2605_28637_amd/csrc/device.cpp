// Device memory layout and the upload of the static tables.
#include <algorithm>
#include <cmath>
#include <cstring>


#include "roks_internal.h"

namespace roks {

// Band pairs per plane-pass workgroup. Each workgroup transforms one z-plane
// for a run of pairs and pays, once per run, a fixed cost about one pair's
// transform (reloading the plane's potentials, or writing its density
// partial). With one such workgroup resident per CU, a pass takes
// ceil(n3 * chunks / cus) rounds of (pairs per chunk + 1); the smallest chunk
// count that minimises that is taken. Fixed per shape and device, so the
// density's chunk sum keeps one order.
static int plane_chunks(int n3, int npairs, int cus) {
  int best = 1;
  long best_cost = -1;
  for (int n = 1; n <= npairs; ++n) {
    const long rounds = cdiv(n3 * n, cus);
    const long cost = rounds * (cdiv(npairs, n) + 1);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = n;
    }
  }
  return best;
}

void ensure_side_stream(Ctx& c) {
  if (c.side) return;
  ROKS_HIP(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
  ROKS_HIP(hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming));
  ROKS_HIP(hipEventCreateWithFlags(&c.ev_join, hipEventDisableTiming));
}

void init_device(Ctx& c, void* stream) {
  int ndev = 0;
  ROKS_CHECK(hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0, ROKS_ERR_HIP, "no HIP device");
  ROKS_HIP(hipGetDevice(&c.device));
  c.stream = reinterpret_cast<hipStream_t>(stream);
  if (!c.stream) {
    // a stream of its own (default priority), so contexts run side by side
    ROKS_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
    c.own_stream = true;
  }
  const size_t nb = c.nb, npw = c.npw, ntot = c.ntot, np = c.nproj;
  // the static scratch of the allocation-free apply on this device
  init_noalloc_scratch(c);
  c.npairs = (c.nb + 1) / 2;
  int cus = 0;
  ROKS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device));
  c.nchunk = plane_chunks(c.N[2], c.npairs, std::max(1, cus));
  if (c.N[0] == c.N[1] && line_split(c.N[0], &c.lines_G, &c.lines_P)) {
    line_split_density(c.N[0], &c.dlines_G, &c.dlines_P);
    // several line-kernel workgroups share a CU: about two rounds of them
    const int n = c.N[0], nh = 2 * c.hmax + 1;
    const size_t lds = (size_t)(n + nh * (n + 1)) * 16 + 1024;
    const int per_cu = std::max(1, std::min(8, (int)((160 * 1024) / lds)));
    c.nchunk = std::max(1, std::min(c.npairs, cdiv(2 * cus * per_cu, c.N[2])));
  } else {
    c.lines_G = c.lines_P = c.dlines_G = c.dlines_P = 0;
  }

  c.d_miller = dalloc<int32_t>(c, 3 * npw);
  c.d_g2 = dalloc<double>(c, npw);
  c.d_cols = dalloc<ColDesc>(c, c.cols.size());
  c.d_colpos = dalloc<int32_t>(c, 2 * (size_t)c.ncol);
  for (int d = 0; d < 3; ++d) {
    c.d_tw[d] = dalloc<double2>(c, c.N[d]);
    c.d_tw32[d] = dalloc<float2>(c, c.N[d]);
  }
  if (c.prec == ROKS_FP32) {
    c.d_vsh32 = dalloc<float>(c, (size_t)c.nsocc * c.ntot);
    c.d_vloc32 = dalloc<float>(c, (size_t)2 * c.nconf * c.ntot);
  }
  c.d_vext = dalloc<double>(c, ntot);
  c.d_B = dalloc<double2>(c, np * npw);
  c.d_proj_atom = dalloc<int32_t>(c, np);
  c.d_Dblk = dalloc<double>(c, c.Dblk.size());
  c.d_Dblk_off = dalloc<int32_t>(c, c.natoms);
  if (c.has_q) c.d_Qblk = dalloc<double>(c, c.Qblk.size());
  c.d_atom_proj_off = dalloc<int32_t>(c, c.natoms);
  c.d_atom_proj_cnt = dalloc<int32_t>(c, c.natoms);
  c.d_band_shell = dalloc<int32_t>(c, nb);
  c.d_atoms = dalloc<char>(c, atom_info_bytes() * std::max(1, c.natoms));
  c.d_projinfo = dalloc<char>(c, proj_info_bytes() * std::max<size_t>(1, np));

  const size_t band = nb * npw;
  c.d_psi = dalloc<double2>(c, band);
  c.d_in = dalloc<double2>(c, band);
  c.d_Y = dalloc<double2>(c, band);
  c.d_gI = dalloc<double2>(c, band);
  if (c.has_q) c.d_Spsi = dalloc<double2>(c, band);
  c.d_p = dalloc<double2>(c, band);
  c.d_S = dalloc<double2>(c, band);
  c.d_Pt = dalloc<double2>(c, band);
  c.d_trial[0] = dalloc<double2>(c, band);
  c.d_trial[1] = dalloc<double2>(c, band);
  // w1 and S_old side by side: one band product covers both (preconditioner)
  c.d_w1 = dalloc<double2>(c, 2 * band);
  c.d_Sold = c.d_w1 + band;
  c.d_T = dalloc<double2>(c, (size_t)c.npairs * c.N[2] * c.ncol);
  c.d_rho_part = dalloc<double>(c, (size_t)c.nchunk * c.nsocc * ntot);
  c.d_rho = dalloc<double>(c, (size_t)c.nsocc * ntot);
  c.d_vloc = dalloc<double>(c, (size_t)2 * c.nconf * ntot);
  c.d_vsh = dalloc<double>(c, (size_t)c.nsocc * ntot);
  c.d_fft = dalloc<double2>(c, ntot);
  c.d_P = dalloc<double>(c, np * nb);
  c.d_DP = dalloc<double>(c, np * nb);
  c.d_dP = dalloc<double>(c, np * nb);
  c.d_P0 = dalloc<double>(c, np * nb);
  c.d_PS = dalloc<double>(c, np * nb);
  c.part_capacity = std::max<size_t>(8 * 1024, (size_t)c.natoms * 32 * 3) + 64;
  c.d_part = dalloc<double>(c, c.part_capacity);
  c.d_scal = dalloc<double>(c, 16 + 2 * nb);
  c.d_red = c.d_scal;
  c.d_kin = c.d_scal + 16;
  c.d_enl = c.d_scal + 16 + nb;
  c.gemm_part_capacity = std::max<size_t>({4 * np * nb, 64 * nb * nb, (size_t)1 << 21});
  c.d_gemm_part = dalloc<double>(c, c.gemm_part_capacity);
  c.d_Qpart = dalloc<double>(c, (size_t)c.npairs * c.N[2] * 2 * c.nsocc);
  c.d_Q = dalloc<double>(c, 2 * (size_t)c.npairs * c.nsocc);
  c.d_bandv = dalloc<double>(c, 8 * nb);
  c.d_cg = dalloc<double>(c, 8 + nb);
  const size_t nn = nb * nb;
  c.d_m12 = dalloc<double>(c, 2 * (size_t)nb * nb);
  double** mats[] = {&c.d_theta, &c.d_R, &c.d_kappa, &c.d_A, &c.d_D, &c.d_Dold, &c.d_gram,
                     &c.d_Linv, &c.d_U, &c.d_M, &c.d_m1, &c.d_m2, &c.d_m3, &c.d_Mkeep,
                     &c.d_Ukeep, &c.d_m4, &c.d_SS, &c.d_PSold};
  for (double** m : mats) *m = dalloc<double>(c, nn);
  if (!expm_in_lds(c)) c.d_ex = dalloc<double>(c, 5 * nn);
  c.d_flag = dalloc<int32_t>(c, 16);
  // the energy sums, step scalars and status flags are written by kernels
  // straight into pinned, coherent host memory (read by the host after a
  // synchronisation; no kernel reads them back), through the device views hd_*
  ROKS_HIP(hipHostMalloc(reinterpret_cast<void**>(&c.h_scal), (16 + 2 * (size_t)nb) * sizeof(double),
                         hipHostMallocMapped | hipHostMallocCoherent));
  ROKS_HIP(hipHostMalloc(reinterpret_cast<void**>(&c.h_stage),
                         (kStage + 4 * (size_t)nb) * sizeof(double),
                         hipHostMallocMapped | hipHostMallocCoherent));
  ROKS_HIP(hipHostMalloc(reinterpret_cast<void**>(&c.h_flag), 16 * sizeof(int32_t),
                         hipHostMallocMapped | hipHostMallocCoherent));
  ROKS_HIP(hipHostMalloc(reinterpret_cast<void**>(&c.h_force),
                         3 * (size_t)std::max(1, c.natoms) * sizeof(double),
                         hipHostMallocMapped | hipHostMallocCoherent));
  ROKS_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c.hd_scal), c.h_scal, 0));
  ROKS_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c.hd_force), c.h_force, 0));
  ROKS_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c.hd_stage), c.h_stage, 0));
  // without projectors the nonlocal band energies stay zero
  std::memset(c.h_scal, 0, (16 + 2 * (size_t)nb) * sizeof(double));
  ROKS_HIP(hipMemsetAsync(c.d_scal, 0, (16 + 2 * (size_t)nb) * sizeof(double), c.stream));
  ROKS_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c.hd_flag), c.h_flag, 0));
  c.d_force = dalloc<double>(c, 3 * (size_t)std::max(1, c.natoms));
  c.d_kinw_shell = dalloc<double>(c, nb);
  c.d_ones = dalloc<double>(c, nb);
  c.d_potidx = dalloc<int32_t>(c, (size_t)6 * nb);
  c.d_kinw_closed = dalloc<double>(c, nb);
}

void upload_static(Ctx& c) {
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (bytes) ROKS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c.stream));
  };
  up(c.d_miller, c.miller.data(), c.miller.size() * sizeof(int32_t));
  up(c.d_g2, c.g2half.data(), c.g2half.size() * sizeof(double));
  up(c.d_cols, c.cols.data(), c.cols.size() * sizeof(ColDesc));
  std::vector<int32_t> colpos(2 * (size_t)c.ncol);
  auto wrap = [](int v, int n) { return ((v % n) + n) % n; };
  for (int j = 0; j <= c.nH; ++j) {
    colpos[2 * j] = wrap(c.cols[j].h, c.N[0]);
    colpos[2 * j + 1] = wrap(c.cols[j].k, c.N[1]);
    if (j > 0) {
      colpos[2 * (c.nH + j)] = wrap(-c.cols[j].h, c.N[0]);
      colpos[2 * (c.nH + j) + 1] = wrap(-c.cols[j].k, c.N[1]);
    }
  }
  up(c.d_colpos, colpos.data(), colpos.size() * sizeof(int32_t));
  // line kernels: LDS position of every column in the pruned plane (row
  // h + hmax, stride N + 1) and the k range of each row, which must be one
  // contiguous run (else the LDS-plane kernels are used)
  if (c.lines_G > 0) {
    const int n = c.N[0], nh = 2 * c.hmax + 1, PS = n + 1;
    std::vector<int32_t> colidx(c.ncol), kr(2 * (size_t)nh);
    std::vector<int32_t> cnt(nh, 0);
    for (int r = 0; r < nh; ++r) {
      kr[2 * r] = 1 << 20;
      kr[2 * r + 1] = -(1 << 20);
    }
    bool ok = true;
    for (int col = 0; col < c.ncol; ++col) {
      int h = colpos[2 * col], k = colpos[2 * col + 1];
      const int hs = 2 * h > n ? h - n : h, ks = 2 * k > n ? k - n : k;
      if (hs < -c.hmax || hs > c.hmax) {
        ok = false;
        break;
      }
      const int r = hs + c.hmax;
      colidx[col] = r * PS + k;
      kr[2 * r] = std::min(kr[2 * r], ks);
      kr[2 * r + 1] = std::max(kr[2 * r + 1], ks);
      cnt[r]++;
    }
    for (int r = 0; ok && r < nh; ++r)
      if (cnt[r] > 0 && cnt[r] != kr[2 * r + 1] - kr[2 * r] + 1) ok = false;
    if (ok) {
      c.d_colidx = dalloc<int32_t>(c, colidx.size());
      c.d_krange = dalloc<int32_t>(c, kr.size());
      up(c.d_colidx, colidx.data(), colidx.size() * sizeof(int32_t));
      up(c.d_krange, kr.data(), kr.size() * sizeof(int32_t));
      ROKS_HIP(hipStreamSynchronize(c.stream));
    } else {
      c.lines_G = c.lines_P = c.dlines_G = c.dlines_P = 0;
    }
  }
  std::vector<double2> tw[3];  // host sources stay alive until the stream synchronises below
  std::vector<float2> tw32[3];
  for (int d = 0; d < 3; ++d) {
    tw[d].resize(c.N[d]);
    tw32[d].resize(c.N[d]);
    for (int k = 0; k < c.N[d]; ++k) {
      long double a = -2.0L * (long double)M_PI * (long double)k / (long double)c.N[d];
      tw[d][k] = make_double2((double)std::cos(a), (double)std::sin(a));
      tw32[d][k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    up(c.d_tw[d], tw[d].data(), tw[d].size() * sizeof(double2));
    up(c.d_tw32[d], tw32[d].data(), tw32[d].size() * sizeof(float2));
  }
  up(c.d_proj_atom, c.proj_atom.data(), c.proj_atom.size() * sizeof(int32_t));
  up(c.d_Dblk, c.Dblk.data(), c.Dblk.size() * sizeof(double));
  up(c.d_Dblk_off, c.Dblk_off.data(), c.Dblk_off.size() * sizeof(int32_t));
  if (c.has_q) up(c.d_Qblk, c.Qblk.data(), c.Qblk.size() * sizeof(double));
  up(c.d_atom_proj_off, c.atom_proj_off.data(), c.atom_proj_off.size() * sizeof(int32_t));
  up(c.d_atom_proj_cnt, c.atom_proj_cnt.data(), c.atom_proj_cnt.size() * sizeof(int32_t));
  up(c.d_band_shell, c.band_shell.data(), c.band_shell.size() * sizeof(int32_t));
  // shell-mode kinetic weights and potential indices; channel-mode indices
  std::vector<double> kw, ones, kwc;
  std::vector<int32_t> pidx;
  kw.assign(c.nb, 0.0);
  ones.assign(c.nb, 1.0);
  kwc.assign(c.nb, 0.0);
  pidx.assign((size_t)6 * c.nb, -1);
  int Xc = -1;
  for (int X = 0; X < c.nshell; ++X)
    if (c.shell_closed[X] && Xc < 0) Xc = X;
  for (int n = 0; n < c.nb; ++n) {
    const int X = c.band_shell[n];
    kw[n] = c.shell_virtual[X] ? 0.0 : c.shell_w[X];
    pidx[n] = c.shell_virtual[X] ? -1 : X;
    for (int ch = 0; ch < 4; ++ch) pidx[(size_t)(1 + ch) * c.nb + n] = ch;
    // row 5: the closed-shell operator F^c for every band
    pidx[(size_t)5 * c.nb + n] = Xc;
    kwc[n] = Xc >= 0 ? c.shell_w[Xc] : 0.0;
  }
  up(c.d_kinw_shell, kw.data(), kw.size() * sizeof(double));
  up(c.d_kinw_closed, kwc.data(), kwc.size() * sizeof(double));
  up(c.d_ones, ones.data(), ones.size() * sizeof(double));
  up(c.d_potidx, pidx.data(), pidx.size() * sizeof(int32_t));
  ROKS_HIP(hipStreamSynchronize(c.stream));
  upload_positions(c);
  ROKS_HIP(hipStreamSynchronize(c.stream));
}

KernelTimer::KernelTimer(Ctx& ctx, const char* name, double bytes, double flops) : c(ctx) {
  if (!c.timing) return;
  if (!c.timing_only.empty() && c.timing_only != name) return;
  Ctx::Timed t;
  t.name = name;
  t.bytes = bytes;
  t.flops = flops;
  if (hipEventCreate(&t.a) != hipSuccess) return;
  if (hipEventCreate(&t.b) != hipSuccess) {
    (void)hipEventDestroy(t.a);
    return;
  }
  if (hipEventRecord(t.a, c.stream) != hipSuccess) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
    return;
  }
  c.timed.push_back(t);
  idx = (int)c.timed.size() - 1;
}

KernelTimer::~KernelTimer() {
  if (idx >= 0) (void)hipEventRecord(c.timed[idx].b, c.stream);
}

void clear_timing(Ctx& c) {
  if (!c.timed.empty()) (void)hipStreamSynchronize(c.stream);
  for (auto& t : c.timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  c.timed.clear();
}

void free_device(Ctx& c) {
  clear_timing(c);
  if (c.stream || !c.allocations.empty()) (void)hipStreamSynchronize(c.stream);
  free_graph_mode(c);
  for (DevBuf& b : c.allocations) (void)hipFree(b.p);
  c.allocations.clear();
  for (void* h : {(void*)c.h_scal, (void*)c.h_stage, (void*)c.h_flag, (void*)c.h_force})
    if (h) (void)hipHostFree(h);
  c.h_scal = c.h_stage = c.h_force = nullptr;
  c.h_flag = nullptr;
  c.hd_scal = c.hd_stage = c.hd_force = nullptr;
  c.hd_flag = nullptr;
  if (c.side) (void)hipStreamSynchronize(c.side);
  if (c.ev_fork) (void)hipEventDestroy(c.ev_fork);
  if (c.ev_join) (void)hipEventDestroy(c.ev_join);
  if (c.side) (void)hipStreamDestroy(c.side);
  c.side = nullptr;
  c.ev_fork = c.ev_join = nullptr;
  if (c.own_stream && c.stream) (void)hipStreamDestroy(c.stream);
  c.stream = nullptr;
  c.own_stream = false;
}

}  // namespace roks
