// C ABI: plan validation, workspace layout and dispatch to the HIP kernels.
#include <new>

#include <hip/hip_runtime.h>

#include "../../include/rgf.h"
#include "kernels.h"

struct rgf_plan_s {
  rgf_desc_t d;
  int bp;
  size_t ws_bytes;
  size_t ws_chain;   // sequential sweep: workspace elements per energy
  // DDRGF workspace layout (byte offsets)
  size_t dd_int_chain, dd_red_chain;
  size_t off_int, off_ms, off_gs, off_gsrow, off_red, off_fin, off_info;
  // w > 1 DDRGF: super-block copies of the inputs and of the output band
  int fl, fb;                    // super-layers and super-block size of the DDRGF system
  size_t off_hf, off_slf, off_srf, off_gf, off_inff;
};

namespace {
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}

namespace {

rgf_status_t validate(const rgf_desc_t* d) {
  if (!d) return RGF_ERR_INVALID_ARG;
  if (d->num_layers < 1 || d->block_size < 1 || d->num_energies < 1 || d->half_bandwidth < 1)
    return RGF_ERR_INVALID_ARG;
  if (d->block_size > 128) return RGF_ERR_UNSUPPORTED;
  if (d->num_layers > 1 && d->half_bandwidth >= d->num_layers) return RGF_ERR_INVALID_ARG;
  if (d->num_layers > (int64_t)1 << 24 || d->num_energies > (int64_t)1 << 24) return RGF_ERR_UNSUPPORTED;
  if (d->precision != RGF_FP64 && d->precision != RGF_MIXED_FP32) return RGF_ERR_UNSUPPORTED;
  // mixed precision: sequential block-tridiagonal sweep only (FP32 products on the
  // closed interiors of DDRGF lose all accuracy on ill-conditioned interiors)
  if (d->precision == RGF_MIXED_FP32 && (d->half_bandwidth > 1 || d->method != RGF_METHOD_SEQUENTIAL))
    return RGF_ERR_UNSUPPORTED;
  if (d->method != RGF_METHOD_SEQUENTIAL && d->method != RGF_METHOD_DDRGF) return RGF_ERR_INVALID_ARG;
  if (d->half_bandwidth > 4) return RGF_ERR_UNSUPPORTED;
  if (d->method == RGF_METHOD_DDRGF) {
    const int64_t w = d->half_bandwidth;
    const int64_t s1 = d->separator_layers == 0 ? w : d->separator_layers;
    if (s1 != w) return RGF_ERR_UNSUPPORTED;
    if (d->num_domains < 1) return RGF_ERR_INVALID_ARG;
    if (d->num_layers - d->num_domains * s1 < d->num_domains * w) return RGF_ERR_INVALID_ARG;
    if (w > 1) {
      // separators of w layers: the w-layer super-block system must fit the kernels
      if (d->num_layers % w != 0 || w * d->block_size > 128) return RGF_ERR_UNSUPPORTED;
      const int64_t lf = d->num_layers / w;
      if (lf - d->num_domains < d->num_domains) return RGF_ERR_INVALID_ARG;
    }
  }
  return RGF_OK;
}

}  // namespace

extern "C" {

rgf_status_t rgf_plan_create(const rgf_desc_t* desc, rgf_plan_t* plan, size_t* workspace_bytes) {
  if (!plan) return RGF_ERR_INVALID_ARG;
  *plan = nullptr;
  rgf_status_t st = validate(desc);
  if (st != RGF_OK) return st;
  rgf_plan_s* p = new (std::nothrow) rgf_plan_s();
  if (!p) return RGF_ERR_OUT_OF_MEMORY;
  p->d = *desc;
  p->bp = rgfk::padded_block((int)desc->block_size);
  const int w = (int)desc->half_bandwidth;
  if (w == 1)
    p->ws_chain = rgfk::sweep_ws_chain_elems((int)desc->num_layers, p->bp);
  else
    p->ws_chain = rgfk::nrgf_ws_chain_elems((int)desc->num_layers, w, p->bp);
  p->ws_bytes = p->ws_chain * sizeof(double2) * (size_t)desc->num_energies;
  if (desc->method == RGF_METHOD_DDRGF) {
    const int l = (int)desc->num_layers / w, m = (int)desc->num_domains, ne = (int)desc->num_energies;
    const size_t b = (size_t)desc->block_size * w, bb = b * b;
    p->fl = l;
    p->fb = (int)b;
    p->bp = rgfk::padded_block((int)b);
    const size_t bpbp = (size_t)p->bp * p->bp;
    int base = 0, rem = 0;
    rgfk::ddrgf_layout_host(l, m, &base, &rem);
    p->dd_int_chain = rgfk::ddrgf_interior_ws_elems(base + 1, p->bp);
    p->dd_red_chain = rgfk::sweep_ws_chain_elems(m, p->bp);
    size_t off = 0;
    p->off_int = off;   off = align256(off + p->dd_int_chain * sizeof(double2) * (size_t)ne * m);
    p->off_ms = off;    off = align256(off + (size_t)ne * 3 * m * bb * sizeof(double2));
    p->off_gs = off;    off = align256(off + (size_t)ne * 3 * m * bb * sizeof(double2));
    p->off_gsrow = off; off = align256(off + (size_t)ne * m * bb * sizeof(double2));
    p->off_red = off;   off = align256(off + p->dd_red_chain * sizeof(double2) * (size_t)ne);
    p->off_fin = off;   off = align256(off + (size_t)ne * 4 * bpbp * sizeof(double2));
    p->off_info = off;  off = align256(off + (size_t)ne * (m + 1) * sizeof(int));
    if (w > 1) {
      p->off_hf = off;   off = align256(off + (size_t)3 * l * bb * sizeof(double2));
      p->off_slf = off;  off = align256(off + (size_t)ne * bb * sizeof(double2));
      p->off_srf = off;  off = align256(off + (size_t)ne * bb * sizeof(double2));
      p->off_gf = off;   off = align256(off + (size_t)ne * 3 * l * bb * sizeof(double2));
      p->off_inff = off; off = align256(off + (size_t)ne * sizeof(int));
    }
    p->ws_bytes = off;
  }
  *plan = p;
  if (workspace_bytes) *workspace_bytes = p->ws_bytes;
  return RGF_OK;
}

rgf_status_t rgf_plan_destroy(rgf_plan_t plan) {
  delete plan;
  return RGF_OK;
}

rgf_status_t rgf_solve(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                       const double* energies, double eta_d, void* G, double* T, int32_t* info,
                       void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return RGF_ERR_INVALID_ARG;
  if (plan->d.method != RGF_METHOD_SEQUENTIAL) return RGF_ERR_PLAN_MISMATCH;
  if (!H || !sigma_L || !sigma_R || !energies || !G || !info) return RGF_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < plan->ws_bytes) return RGF_ERR_WORKSPACE_TOO_SMALL;
  const rgf_desc_t& d = plan->d;
  if (d.half_bandwidth > 1) {
    rgfk::NSweepArgs n{};
    n.H = static_cast<const double2*>(H);
    n.sigL = static_cast<const double2*>(sigma_L);
    n.sigR = static_cast<const double2*>(sigma_R);
    n.E = energies;
    n.eta_d = eta_d;
    n.G = static_cast<double2*>(G);
    n.T = d.want_transmission ? T : nullptr;
    n.info = info;
    n.ws = static_cast<double2*>(workspace);
    n.ws_chain = plan->ws_chain;
    n.l = (int)d.num_layers;
    n.b = (int)d.block_size;
    n.w = (int)d.half_bandwidth;
    n.ne = (int)d.num_energies;
    hipError_t e = rgfk::launch_nrgf_sweep(n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RGF_OK : RGF_ERR_HIP;
  }
  rgfk::SweepArgs a{};
  a.H = static_cast<const double2*>(H);
  a.h_stride = 0;
  a.sigL = static_cast<const double2*>(sigma_L);
  a.sigR = static_cast<const double2*>(sigma_R);
  a.E = energies;
  a.eta_d = eta_d;
  a.direct = 0;
  a.G = static_cast<double2*>(G);
  a.g_stride = (size_t)3 * d.num_layers * d.block_size * d.block_size;
  a.first_row = nullptr;
  a.T = d.want_transmission ? T : nullptr;
  a.info = info;
  a.info_stride = 1;
  a.info_offset = 0;
  a.ws = static_cast<double2*>(workspace);
  a.ws_chain = plan->ws_chain;
  a.l = (int)d.num_layers;
  a.b = (int)d.block_size;
  a.chains = (int)d.num_energies;
  a.mixed = d.precision == RGF_MIXED_FP32 ? 1 : 0;
  hipError_t e = rgfk::launch_rgf_sweep(a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? RGF_OK : RGF_ERR_HIP;
}

rgf_status_t ddrgf_solve(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                         const double* energies, double eta_d, void* G, double* T, int32_t* info,
                         void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return RGF_ERR_INVALID_ARG;
  if (plan->d.method != RGF_METHOD_DDRGF) return RGF_ERR_PLAN_MISMATCH;
  if (!H || !sigma_L || !sigma_R || !energies || !G || !info) return RGF_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < plan->ws_bytes) return RGF_ERR_WORKSPACE_TOO_SMALL;
  const rgf_desc_t& d = plan->d;
  char* ws = static_cast<char*>(workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int w = (int)d.half_bandwidth;
  rgfk::FuseArgs f{};
  if (w > 1) {
    f.H = static_cast<const double2*>(H);
    f.sigL = static_cast<const double2*>(sigma_L);
    f.sigR = static_cast<const double2*>(sigma_R);
    f.Hf = reinterpret_cast<double2*>(ws + plan->off_hf);
    f.sigLf = reinterpret_cast<double2*>(ws + plan->off_slf);
    f.sigRf = reinterpret_cast<double2*>(ws + plan->off_srf);
    f.Gf = reinterpret_cast<double2*>(ws + plan->off_gf);
    f.G = static_cast<double2*>(G);
    f.info_f = reinterpret_cast<int*>(ws + plan->off_inff);
    f.info = info;
    f.l = (int)d.num_layers;
    f.b = (int)d.block_size;
    f.w = w;
    f.ne = (int)d.num_energies;
    if (rgfk::launch_fuse(f, st) != hipSuccess) return RGF_ERR_HIP;
  }
  rgfk::DDArgs a{};
  a.H = w > 1 ? f.Hf : static_cast<const double2*>(H);
  a.sigL = w > 1 ? f.sigLf : static_cast<const double2*>(sigma_L);
  a.sigR = w > 1 ? f.sigRf : static_cast<const double2*>(sigma_R);
  a.E = energies;
  a.eta_d = eta_d;
  a.G = w > 1 ? const_cast<double2*>(f.Gf) : static_cast<double2*>(G);
  a.T = d.want_transmission ? T : nullptr;
  a.info = w > 1 ? const_cast<int*>(f.info_f) : info;
  a.l = plan->fl;
  a.b = plan->fb;
  a.m = (int)d.num_domains;
  a.ne = (int)d.num_energies;
  a.ws_int = reinterpret_cast<double2*>(ws + plan->off_int);
  a.ws_int_chain = plan->dd_int_chain;
  a.MS = reinterpret_cast<double2*>(ws + plan->off_ms);
  a.GS = reinterpret_cast<double2*>(ws + plan->off_gs);
  a.GSrow = reinterpret_cast<double2*>(ws + plan->off_gsrow);
  a.ws_red = reinterpret_cast<double2*>(ws + plan->off_red);
  a.ws_red_chain = plan->dd_red_chain;
  a.ws_fin = reinterpret_cast<double2*>(ws + plan->off_fin);
  a.info_part = reinterpret_cast<int*>(ws + plan->off_info);
  a.mixed = d.precision == RGF_MIXED_FP32 ? 1 : 0;
  hipError_t e = rgfk::launch_ddrgf(a, st);
  if (e == hipSuccess && w > 1) e = rgfk::launch_unfuse(f, st);
  return e == hipSuccess ? RGF_OK : RGF_ERR_HIP;
}

const char* rgf_status_string(rgf_status_t s) {
  switch (s) {
    case RGF_OK: return "ok";
    case RGF_ERR_INVALID_ARG: return "invalid argument";
    case RGF_ERR_UNSUPPORTED: return "unsupported configuration";
    case RGF_ERR_OUT_OF_MEMORY: return "out of host memory";
    case RGF_ERR_WORKSPACE_TOO_SMALL: return "workspace missing or too small";
    case RGF_ERR_HIP: return "HIP runtime error";
    case RGF_ERR_PLAN_MISMATCH: return "plan does not match the entry point";
  }
  return "unknown status";
}

int rgf_version(void) { return 100; }

}  // extern "C"
