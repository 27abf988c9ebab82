// Host side of the diagnostics sweep and its entry point. Included once by
// fe_api.hip.
#pragma once

namespace {

// The diagnostics sweep: one tile shape for both precisions.
constexpr int kDiagTX = 64, kDiagTY = 8, kDiagNT = 512;

template <typename T>
int diagnostics(fe_ctx* c, const void* u, void* curv, double* hist, int nbins, double kmax, double* stats) {
  const int B = c->grid.batch;
  const int ntx = ceil_div(c->grid.nx, kDiagTX), nty = ceil_div(c->grid.ny, kDiagTY);
  // z chunks by the makespan model: at 256^3 in FP32, 43-plane chunks give 768
  // blocks, one round of three per CU, where 32-plane chunks gave 1024 blocks and
  // a last round a third full
  int slots = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&slots, (const void*)fe::diag_sweep<T, kDiagTX, kDiagTY, kDiagNT>,
                                                   kDiagNT, 0) != hipSuccess ||
      slots < 1)
    slots = 1;
  const int lz = halo1_chunk((long)ntx * nty * B, c->grid.nz, c->num_cu, slots);
  const int nzc = ceil_div(c->grid.nz, lz);
  const size_t per_inst = (size_t)ntx * nty * nzc;
  // layout of d_diag: DiagInst[B] | stats[B][5] | partials[B][per_inst][5]
  const size_t need = sizeof(fe::DiagInst) * B + sizeof(double) * fe::kDiagStats * B * (1 + per_inst);
  if (c->diag_bytes < need) {
    if (c->d_diag) (void)hipFree(c->d_diag);
    c->d_diag = nullptr;
    c->diag_bytes = 0;
    if (hipMalloc((void**)&c->d_diag, need) != hipSuccess) {
      c->d_diag = nullptr;
      return set_error(FE_ENOMEM, "diagnostics workspace allocation failed");
    }
    c->diag_bytes = need;
  }
  const double h = c->grid.h;
  std::vector<fe::DiagInst> di(B);
  for (int b = 0; b < B; ++b) {
    const double eps = c->eps[b];
    di[b] = fe::DiagInst{eps * h / 8.0, h * h * h / (4.0 * eps), eps * h / 4.0};
  }
  fe::DiagInst* d_inst = reinterpret_cast<fe::DiagInst*>(c->d_diag);
  double* d_stats = reinterpret_cast<double*>(d_inst + B);
  double* d_part = d_stats + (size_t)fe::kDiagStats * B;
  FE_HIP(hipMemcpyAsync(d_inst, di.data(), sizeof(fe::DiagInst) * B, hipMemcpyHostToDevice, c->stream));
  if (hist) {
    const int n = B * nbins * nbins;
    hipLaunchKernelGGL(fe::fill_f64, dim3(ceil_div(n, 64)), dim3(64), 0, c->stream, hist, n, 0.0);
  }
  fe::SweepArgs<T> a{};
  a.src = static_cast<const T*>(u);
  a.prm = static_cast<const fe::InstParams<T>*>(c->d_prm);
  a.cfield = c->use_cfield ? static_cast<const T*>(c->d_cfield) : nullptr;
  a.k = grid_consts<T>(h);
  a.nx = c->grid.nx;
  a.ny = c->grid.ny;
  a.nz = c->grid.nz;
  a.ntx = ntx;
  a.nty = nty;
  a.nzc = nzc;
  a.lz = lz;
  a.batch = B;
  fe::DiagArgs<T> d{};
  d.inst = d_inst;
  d.curv = static_cast<T*>(curv);
  d.hist = hist;
  d.partials = d_part;
  d.nbins = hist ? nbins : 0;
  d.kmax = T(kmax);
  d.bin_scale = T(hist ? nbins / (2.0 * kmax) : 0.0);
  d.inv_h = T(1.0 / h);
  d.inv_h2 = T(1.0 / (h * h));
  hipLaunchKernelGGL((fe::diag_sweep<T, kDiagTX, kDiagTY, kDiagNT>), dim3((unsigned)(per_inst * B)),
                     dim3(kDiagNT), 0, c->stream, a, d);
  hipLaunchKernelGGL(fe::diag_finish, dim3(B), dim3(256), 0, c->stream, (const double*)d_part, (int)per_inst,
                     d_stats);
  FE_HIP(hipGetLastError());
  if (stats) {
    FE_HIP(hipMemcpyAsync(stats, d_stats, sizeof(double) * fe::kDiagStats * B, hipMemcpyDeviceToHost, c->stream));
    FE_HIP(hipStreamSynchronize(c->stream));
  }
  return FE_OK;
}

}  // namespace

extern "C" {

int fe_diagnostics(fe_ctx* c, const void* u, void* curv, double* hist, int nbins, double kmax, double* stats) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!u) return set_error(FE_EINVAL, "u is NULL");
  if (curv == u) return set_error(FE_EINVAL, "curv must not alias u");
  if (hist) {
    if (nbins < 1 || nbins > fe::kDiagMaxBins)
      return set_error(FE_EINVAL, "nbins must lie in [1, %d] (got %d)", fe::kDiagMaxBins, nbins);
    if (!(kmax > 0.0) || !std::isfinite(kmax)) return set_error(FE_EINVAL, "kmax must be finite and > 0");
  }
  DeviceGuard dg(c->device);
  return c->grid.dtype == FE_F32 ? diagnostics<float>(c, u, curv, hist, nbins, kmax, stats)
                                 : diagnostics<double>(c, u, curv, hist, nbins, kmax, stats);
}

}  // extern "C"
