// C ABI: plan validation, workspace layout and dispatch to the HIP kernels.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/rgf.h"
#include "epilogue.h"
#include "kernels.h"
#include "nlesser.h"

struct rgf_plan_s {
  rgf_desc_t d;
  int bp;
  size_t ws_bytes;
  size_t ws_chain;   // sequential sweep: workspace elements per energy
  // adjoint (want_backward): checkpoint domains, energy chunks; the workspace starts
  // with the checkpoints (ck_bytes, preserved from rgf_solve to rgf_backward) and the
  // rest is scratch shared by the forward sweep and the adjoint
  int nd = 0, dlen = 0, nch = 0;
  size_t ck_chain = 0, ck_bytes = 0, off_fwd = 0, off_adj = 0, adj_wg = 0, off_grad = 0, off_hpart = 0;
  // split sweep (several workgroups per energy): group counters at off_sync (plain
  // sequential w = 1 plans); the requested and the resolved workgroups per energy
  size_t off_sync = 0;
  int split_want = 0, split_k = -1, split_dev = -1, split_used = 1;
  long long split_spin = 0;
  // DDRGF workspace layout (byte offsets)
  size_t dd_int_chain, dd_red_chain;
  size_t off_int, off_ms, off_gs, off_gsrow, off_red, off_fin, off_info, off_herm;
  // second DDRGF level (inner_domains > 0): its interiors, reduced band, inverse band and
  // first row, sweep workspace, finalize scratch, status, and the inner form of the band
  size_t dd2_int_chain = 0, dd2_red_chain = 0;
  size_t off2_int = 0, off2_ms = 0, off2_gs = 0, off2_gsrow = 0, off2_red = 0, off2_fin = 0, off2_info = 0,
         off2_band = 0;
  // w > 1 DDRGF, native form: per (energy, interior) chains, reduced band (half bandwidth
  // 2w - 1 over the m w separator layers) and its inverse, the inverse's first w rows at
  // the last column, the reduced sweep's workspace, finalize scratch, status
  int ndd = 0;
  size_t nd_int_chain = 0, nd_red_chain = 0;
  size_t offn_int = 0, offn_ms = 0, offn_gs = 0, offn_gslast = 0, offn_red = 0, offn_fin = 0, offn_info = 0,
         offn_infored = 0, offn_herm = 0, offn_sync = 0;
  // w > 1 DDRGF, super-block form: copies of the inputs and of the output band
  int fl, fb;                    // super-layers and super-block size of the DDRGF system
  size_t off_hf, off_slf, off_srf, off_gf, off_inff;
  // batched plans
  int batched = 0;
  std::vector<rgf_batch_shape_t> shapes;
  int n_items = 0, grid = 0, waves = 8;
  int* d_index = nullptr;        // device: queue[n], inst_dev[n], inst_energy[n], shape[n_dev][2]
  size_t ws_slot = 0;
  std::mutex mu;                 // guards the cached graph
  bool has_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* g_devs = nullptr;
  void* g_ws = nullptr;
  double g_eta = 0.0;
  hipStream_t g_stream = nullptr;
  // per-kernel timing: event pool, the kernel each event closes (nullptr = the
  // solve's start mark), marks used and dropped since the last query
  bool timing = false;
  std::vector<hipEvent_t> tev;
  std::vector<const char*> tname;
  int tused = 0, tdropped = 0;
};

namespace {
// plan whose solve is being queued on this host thread, when it is timed
thread_local rgf_plan_s* t_timed = nullptr;

void record_mark(rgf_plan_s* p, const char* name, hipStream_t s) {
  if (p->tused >= (int)p->tev.size()) {
    ++p->tdropped;
    return;
  }
  if (hipEventRecord(p->tev[p->tused], s) != hipSuccess) {
    ++p->tdropped;
    return;
  }
  p->tname[p->tused++] = name;
}

// Marks the start of a solve and routes the launchers' marks to the plan.
struct TimedScope {
  explicit TimedScope(rgf_plan_s* p, hipStream_t s) {
    if (p->timing) {
      t_timed = p;
      record_mark(p, nullptr, s);
    }
  }
  ~TimedScope() { t_timed = nullptr; }
};
}  // namespace

namespace rgfk {
void ktime_mark(const char* kernel, hipStream_t s) {
  if (t_timed) record_mark(t_timed, kernel, s);
}
}  // namespace rgfk

namespace {
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr double DEFAULT_MIXED_TOLERANCE = 1e-5;
constexpr int ADJOINT_ENERGY_CHUNKS = 64;
constexpr long long DEFAULT_SPLIT_SPIN = 1LL << 22;
// largest pivot kappa_1 with FP32 products: tolerance / 2^-24
double kappa_limit(double tol) { return (tol > 0.0 ? tol : DEFAULT_MIXED_TOLERANCE) * 16777216.0; }
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
  if (!(d->mixed_tolerance >= 0.0)) return RGF_ERR_INVALID_ARG;
  // mixed precision: sequential block-tridiagonal sweep only (FP32 products on the
  // closed interiors of DDRGF lose all accuracy on ill-conditioned interiors)
  if (d->precision == RGF_MIXED_FP32 && (d->half_bandwidth > 1 || d->method != RGF_METHOD_SEQUENTIAL))
    return RGF_ERR_UNSUPPORTED;
  if (d->method != RGF_METHOD_SEQUENTIAL && d->method != RGF_METHOD_DDRGF) return RGF_ERR_INVALID_ARG;
  if (d->half_bandwidth > 4) return RGF_ERR_UNSUPPORTED;
  if (d->want_backward) {
    if (d->want_backward & ~(RGF_BACKWARD_ONSITE | RGF_BACKWARD_BAND)) return RGF_ERR_INVALID_ARG;
    if (d->method != RGF_METHOD_SEQUENTIAL || d->half_bandwidth != 1 || d->precision != RGF_FP64)
      return RGF_ERR_UNSUPPORTED;
    if (d->checkpoint_domains < 0) return RGF_ERR_INVALID_ARG;
  }
  if (d->inner_domains != 0) {
    if (d->inner_domains < 0 || d->method != RGF_METHOD_DDRGF) return RGF_ERR_INVALID_ARG;
    if (d->precision != RGF_FP64) return RGF_ERR_UNSUPPORTED;
    if (d->num_domains < 2 * d->inner_domains) return RGF_ERR_INVALID_ARG;
  }
  if (d->method == RGF_METHOD_DDRGF) {
    const int64_t w = d->half_bandwidth;
    const int64_t s1 = d->separator_layers == 0 ? w : d->separator_layers;
    if (s1 != w) return RGF_ERR_UNSUPPORTED;
    if (d->num_domains < 1) return RGF_ERR_INVALID_ARG;
    if (d->num_layers - d->num_domains * s1 < d->num_domains * w) return RGF_ERR_INVALID_ARG;
    if (d->ddrgf_form != 0 && d->ddrgf_form != 1) return RGF_ERR_INVALID_ARG;
    if (w == 1 && d->ddrgf_form != 0) return RGF_ERR_INVALID_ARG;
    if (w > 1 && d->ddrgf_form == 0 && d->inner_domains != 0) return RGF_ERR_UNSUPPORTED;
    if (w > 1 && d->ddrgf_form == 1) {
      // separators of w layers: the w-layer super-block system must fit the kernels
      if (d->num_layers % w != 0 || w * d->block_size > 128) return RGF_ERR_UNSUPPORTED;
      const int64_t lf = d->num_layers / w;
      if (lf - d->num_domains < d->num_domains) return RGF_ERR_INVALID_ARG;
    }
  } else if (d->ddrgf_form != 0) {
    return RGF_ERR_INVALID_ARG;
  }
  return RGF_OK;
}

// Workgroups per energy for a plain sequential solve on this stream's device.
int split_for(rgf_plan_s* p, hipStream_t st) {
  const rgf_desc_t& d = p->d;
  if (d.method != RGF_METHOD_SEQUENTIAL || d.precision != RGF_FP64 || d.want_backward || p->split_want == 1)
    return 1;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return 1;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  std::lock_guard<std::mutex> lock(p->mu);
  if (p->split_k < 0 || p->split_dev != dev) {
    p->split_k = d.half_bandwidth == 1
                     ? rgfk::split_workgroups((int)d.block_size, (int)d.num_energies, p->split_want)
                     : rgfk::split_workgroups_n((int)d.block_size, (int)d.num_energies, p->split_want);
    p->split_dev = dev;
  }
  return p->split_k;
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
  else  // + the lesser function's 2w last-column transfer blocks
    p->ws_chain = rgfk::nrgf_ws_chain_elems((int)desc->num_layers, w, p->bp) + (size_t)2 * w * p->bp * p->bp;
  p->ws_bytes = p->ws_chain * sizeof(double2) * (size_t)desc->num_energies;
  if (desc->method == RGF_METHOD_SEQUENTIAL && !desc->want_backward) {
    // group counters of the split sweep, 64 bytes per energy
    p->off_sync = align256(p->ws_bytes);
    p->ws_bytes = p->off_sync + (size_t)64 * desc->num_energies;
  }
  if (desc->want_backward) {
    const int l = (int)desc->num_layers, ne = (int)desc->num_energies, b = (int)desc->block_size;
    const size_t bpbp = (size_t)p->bp * p->bp;
    const int req = desc->checkpoint_domains > 0 ? (int)std::min<int64_t>(desc->checkpoint_domains, l) : std::min(8, l);
    p->dlen = (l + req - 1) / req;
    p->nd = (l + p->dlen - 1) / p->dlen;
    // energy chunks of the adjoint: a function of nE only, so that the band gradient's
    // summation order does not depend on the number of domains
    p->nch = std::min(ne, ADJOINT_ENERGY_CHUNKS);
    p->ck_chain = (size_t)(4 * p->nd + 1) * bpbp;
    p->ck_bytes = align256(p->ck_chain * sizeof(double2) * (size_t)ne);
    p->off_fwd = p->ck_bytes;
    const size_t fwd = p->ws_chain * sizeof(double2) * (size_t)ne;
    p->adj_wg = rgfk::adjoint_scratch_wg_elems(p->dlen, p->bp);
    p->off_adj = p->ck_bytes;
    p->off_grad = align256(p->off_adj + p->adj_wg * sizeof(double2) * (size_t)p->nd * p->nch);
    p->off_hpart = align256(p->off_grad + (size_t)ne * l * b * sizeof(double));
    size_t adj_end = p->off_hpart;
    if (desc->want_backward & RGF_BACKWARD_BAND) adj_end += (size_t)p->nch * 3 * l * (size_t)b * b * sizeof(double2);
    p->ws_bytes = align256(std::max(p->off_fwd + fwd, adj_end));
  }
  if (desc->method == RGF_METHOD_DDRGF && w > 1 && desc->ddrgf_form == 0) {
    const int l = (int)desc->num_layers, m = (int)desc->num_domains, ne = (int)desc->num_energies;
    const int lr = m * w, wr = 2 * w - 1;
    const size_t b = (size_t)desc->block_size, bb = b * b, bpbp = (size_t)p->bp * p->bp;
    int base = 0, rem = 0;
    rgfk::nddrgf_layout_host(l, m, w, &base, &rem);
    p->ndd = 1;
    p->nd_int_chain = rgfk::nddrgf_interior_ws_elems(base + 1, w, p->bp);
    p->nd_red_chain = rgfk::nrgf_ws_chain_elems(lr, wr, p->bp, w);
    const size_t red_band = (size_t)(2 * wr + 1) * lr * bb * sizeof(double2) * ne;
    size_t off = 0;
    p->offn_int = off;     off = align256(off + p->nd_int_chain * sizeof(double2) * (size_t)ne * m);
    p->offn_ms = off;      off = align256(off + red_band);
    p->offn_gs = off;      off = align256(off + red_band);
    p->offn_gslast = off;  off = align256(off + (size_t)ne * w * bb * sizeof(double2));
    p->offn_red = off;     off = align256(off + p->nd_red_chain * sizeof(double2) * (size_t)ne);
    p->offn_fin = off;     off = align256(off + (size_t)ne * 4 * bpbp * sizeof(double2));
    p->offn_info = off;    off = align256(off + (size_t)ne * m * sizeof(int));
    p->offn_infored = off; off = align256(off + (size_t)ne * sizeof(int));
    p->offn_herm = off;    off = align256(off + sizeof(int));
    p->offn_sync = off;    off = align256(off + (size_t)64 * ne);
    p->ws_bytes = off;
  } else if (desc->method == RGF_METHOD_DDRGF) {
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
    p->off_herm = off;  off = align256(off + sizeof(int));
    if (desc->inner_domains > 0) {
      const int m2 = (int)desc->inner_domains;
      int base2 = 0, rem2 = 0;
      rgfk::ddrgf_layout_host(m, m2, &base2, &rem2);
      p->dd2_int_chain = rgfk::ddrgf_interior_ws_elems(base2 + 1, p->bp);
      p->dd2_red_chain = rgfk::sweep_ws_chain_elems(m2, p->bp);
      p->off2_int = off;   off = align256(off + p->dd2_int_chain * sizeof(double2) * (size_t)ne * m2);
      p->off2_ms = off;    off = align256(off + (size_t)ne * 3 * m2 * bb * sizeof(double2));
      p->off2_gs = off;    off = align256(off + (size_t)ne * 3 * m2 * bb * sizeof(double2));
      p->off2_gsrow = off; off = align256(off + (size_t)ne * m2 * bb * sizeof(double2));
      p->off2_red = off;   off = align256(off + p->dd2_red_chain * sizeof(double2) * (size_t)ne);
      p->off2_fin = off;   off = align256(off + (size_t)ne * 4 * bpbp * sizeof(double2));
      p->off2_info = off;  off = align256(off + (size_t)ne * (m2 + 1) * sizeof(int));
      p->off2_band = off;  off = align256(off + (size_t)ne * 3 * m * bb * sizeof(double2));
    }
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
  if (!plan) return RGF_OK;
  if (plan->has_graph) {
    hipGraphExecDestroy(plan->exec);
    hipGraphDestroy(plan->graph);
  }
  if (plan->d_index) hipFree(plan->d_index);
  for (hipEvent_t ev : plan->tev) hipEventDestroy(ev);
  delete plan;
  return RGF_OK;
}

rgf_status_t rgf_batched_plan_create(int64_t num_devices, const rgf_batch_shape_t* shapes,
                                     int32_t precision, int32_t schedule, int32_t grid, int32_t waves,
                                     rgf_plan_t* plan, size_t* workspace_bytes) {
  if (!plan) return RGF_ERR_INVALID_ARG;
  *plan = nullptr;
  if (num_devices < 1 || num_devices > (1 << 20) || !shapes) return RGF_ERR_INVALID_ARG;
  if (precision != RGF_FP64 && precision != RGF_MIXED_FP32) return RGF_ERR_UNSUPPORTED;
  if (schedule < 0 || schedule > 2 || grid < 0) return RGF_ERR_INVALID_ARG;
  if (waves != 0 && waves != 4 && waves != 8) return RGF_ERR_INVALID_ARG;
  struct Item { int dev, en; double cost; int b; };
  std::vector<Item> items;
  size_t slot = 0;
  for (int64_t d = 0; d < num_devices; ++d) {
    const rgf_batch_shape_t& sh = shapes[d];
    if (sh.num_layers < 1 || sh.num_layers > (1 << 20) || sh.num_energies < 1 || sh.num_energies > (1 << 20))
      return RGF_ERR_INVALID_ARG;
    if (sh.block_size < 1) return RGF_ERR_INVALID_ARG;
    if (sh.block_size > 128) return RGF_ERR_UNSUPPORTED;
    slot = std::max(slot, rgfk::sweep_ws_chain_elems((int)sh.num_layers, rgfk::padded_block((int)sh.block_size)));
    const double cost = (double)sh.num_layers * (double)sh.block_size * sh.block_size * sh.block_size;
    for (int64_t e = 0; e < sh.num_energies; ++e) items.push_back({(int)d, (int)e, cost, (int)sh.block_size});
  }
  if (items.size() > (size_t)1 << 30) return RGF_ERR_UNSUPPORTED;
  if (schedule == RGF_SCHEDULE_LONGEST_FIRST) {
    std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
  } else if (schedule == RGF_SCHEDULE_INTERLEAVED) {
    // longest first inside each block size, then take one from each size in turn
    std::vector<std::vector<Item>> by(8);
    for (const Item& it : items) by[rgfk::padded_block(it.b) / 16 - 1].push_back(it);
    for (auto& v : by)
      std::stable_sort(v.begin(), v.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
    std::vector<size_t> pos(8, 0);
    items.clear();
    for (bool more = true; more;) {
      more = false;
      for (int c = 7; c >= 0; --c)
        if (pos[c] < by[c].size()) {
          items.push_back(by[c][pos[c]++]);
          more = true;
        }
    }
  }
  const int n = (int)items.size();
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RGF_ERR_HIP;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return RGF_ERR_HIP;
  const int g = std::max(1, std::min(grid > 0 ? grid : cus, n));
  std::vector<int> host(3 * (size_t)n + 2 * (size_t)num_devices);
  for (int k = 0; k < n; ++k) {
    host[k] = k;                       // instance id = queue position: the tables are in queue order
    host[n + k] = items[k].dev;
    host[2 * n + k] = items[k].en;
  }
  for (int64_t d = 0; d < num_devices; ++d) {
    host[3 * (size_t)n + 2 * d] = (int)shapes[d].num_layers;
    host[3 * (size_t)n + 2 * d + 1] = (int)shapes[d].block_size;
  }
  rgf_plan_s* p = new (std::nothrow) rgf_plan_s();
  if (!p) return RGF_ERR_OUT_OF_MEMORY;
  p->batched = 1;
  p->d = rgf_desc_t{};
  p->d.precision = precision;
  p->shapes.assign(shapes, shapes + num_devices);
  p->n_items = n;
  p->waves = waves == 0 ? 8 : waves;
  p->grid = waves == 4 && grid == 0 ? std::max(1, std::min(2 * cus, n)) : g;
  p->ws_slot = slot;
  if (hipMalloc(&p->d_index, host.size() * sizeof(int)) != hipSuccess) {
    delete p;
    return RGF_ERR_OUT_OF_MEMORY;
  }
  if (hipMemcpy(p->d_index, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(p->d_index);
    delete p;
    return RGF_ERR_HIP;
  }
  p->ws_bytes = 256 + (size_t)g * slot * sizeof(double2);
  *plan = p;
  if (workspace_bytes) *workspace_bytes = p->ws_bytes;
  return RGF_OK;
}

rgf_status_t rgf_batched_solve(rgf_plan_t plan, const rgf_batch_device_t* devices, double eta_d,
                               void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan || !plan->batched) return plan ? RGF_ERR_PLAN_MISMATCH : RGF_ERR_INVALID_ARG;
  if (!devices) return RGF_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < plan->ws_bytes) return RGF_ERR_WORKSPACE_TOO_SMALL;
  char* ws = static_cast<char*>(workspace);
  rgfk::BatchArgs a{};
  a.devs = devices;
  a.queue = plan->d_index;
  a.inst_dev = plan->d_index + plan->n_items;
  a.inst_energy = plan->d_index + 2 * (size_t)plan->n_items;
  a.dev_shape = plan->d_index + 3 * (size_t)plan->n_items;
  a.n_items = plan->n_items;
  a.counter = reinterpret_cast<int*>(ws);
  a.ws_slots = reinterpret_cast<double2*>(ws + 256);
  a.ws_slot = plan->ws_slot;
  a.eta_d = eta_d;
  a.mixed = plan->d.precision == RGF_MIXED_FP32 ? 1 : 0;
  a.kappa_max = kappa_limit(0.0);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (st == nullptr) {
    // the default stream cannot be captured: launch directly
    return rgfk::launch_rgf_batched(a, plan->grid, plan->waves, st) == hipSuccess ? RGF_OK : RGF_ERR_HIP;
  }
  std::lock_guard<std::mutex> lock(plan->mu);
  const bool same = plan->has_graph && plan->g_devs == devices && plan->g_ws == workspace &&
                    plan->g_eta == eta_d && plan->g_stream == st;
  if (!same) {
    if (plan->has_graph) {
      hipGraphExecDestroy(plan->exec);
      hipGraphDestroy(plan->graph);
      plan->has_graph = false;
    }
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      return rgfk::launch_rgf_batched(a, plan->grid, plan->waves, st) == hipSuccess ? RGF_OK : RGF_ERR_HIP;
    }
    hipError_t le = rgfk::launch_rgf_batched(a, plan->grid, plan->waves, st);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(st, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      return RGF_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      hipGraphDestroy(graph);
      return RGF_ERR_HIP;
    }
    plan->graph = graph;
    plan->exec = exec;
    plan->has_graph = true;
    plan->g_devs = devices;
    plan->g_ws = workspace;
    plan->g_eta = eta_d;
    plan->g_stream = st;
  }
  return hipGraphLaunch(plan->exec, st) == hipSuccess ? RGF_OK : RGF_ERR_HIP;
}

rgf_status_t rgf_solve(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                       const double* energies, double eta_d, void* G, double* T, int32_t* info,
                       void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return RGF_ERR_INVALID_ARG;
  if (plan->batched || plan->d.method != RGF_METHOD_SEQUENTIAL) return RGF_ERR_PLAN_MISMATCH;
  if (!H || !sigma_L || !sigma_R || !energies || !G || !info) return RGF_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < plan->ws_bytes) return RGF_ERR_WORKSPACE_TOO_SMALL;
  const rgf_desc_t& d = plan->d;
  TimedScope timed(plan, static_cast<hipStream_t>(stream));
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
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int K = split_for(plan, st);
    if (K > 1) {
      n.sync = reinterpret_cast<unsigned*>(static_cast<char*>(workspace) + plan->off_sync);
      n.spin_limit = plan->split_spin > 0 ? plan->split_spin : DEFAULT_SPLIT_SPIN;
      if (rgfk::launch_nrgf_split(n, K, st) == hipSuccess) {
        plan->split_used = K;
        return RGF_OK;
      }
      (void)hipGetLastError();
    }
    plan->split_used = 1;
    hipError_t e = rgfk::launch_nrgf_sweep(n, st);
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
  a.ws = reinterpret_cast<double2*>(static_cast<char*>(workspace) + plan->off_fwd);
  a.ws_chain = plan->ws_chain;
  a.ck = d.want_backward ? static_cast<double2*>(workspace) : nullptr;
  a.ck_chain = plan->ck_chain;
  a.l = (int)d.num_layers;
  a.b = (int)d.block_size;
  a.chains = (int)d.num_energies;
  a.mixed = d.precision == RGF_MIXED_FP32 ? 1 : 0;
  a.kappa_max = kappa_limit(d.mixed_tolerance);
  a.nd = d.want_backward ? plan->nd : 0;
  a.dlen = d.want_backward ? plan->dlen : 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int K = split_for(plan, st);
  if (K > 1) {
    a.sync = reinterpret_cast<unsigned*>(static_cast<char*>(workspace) + plan->off_sync);
    a.spin_limit = plan->split_spin > 0 ? plan->split_spin : DEFAULT_SPLIT_SPIN;
    hipError_t e = rgfk::launch_rgf_split(a, K, st);
    if (e == hipSuccess) {
      plan->split_used = K;
      return RGF_OK;
    }
    // not launchable right now (e.g. the cooperative grid does not fit): one
    // workgroup per energy instead
    (void)hipGetLastError();
  }
  plan->split_used = 1;
  hipError_t e = rgfk::launch_rgf_sweep(a, st);
  return e == hipSuccess ? RGF_OK : RGF_ERR_HIP;
}

rgf_status_t rgf_solve_lesser(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                              const double* energies, double eta_d, const double* occupation_L,
                              const double* occupation_R, void* G, void* G_lesser, double* T, int32_t* info,
                              void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return RGF_ERR_INVALID_ARG;
  if (plan->batched || plan->d.method != RGF_METHOD_SEQUENTIAL) return RGF_ERR_PLAN_MISMATCH;
  const rgf_desc_t& d = plan->d;
  if (d.precision != RGF_FP64 || d.want_backward) return RGF_ERR_UNSUPPORTED;
  if (!occupation_L || !occupation_R || !G_lesser) return RGF_ERR_INVALID_ARG;
  rgf_status_t st = rgf_solve(plan, H, sigma_L, sigma_R, energies, eta_d, G, T, info, workspace,
                              workspace_bytes, stream);
  if (st != RGF_OK) return st;
  TimedScope timed(plan, static_cast<hipStream_t>(stream));
  rgfk::LesserArgs a{};
  a.sigL = static_cast<const double2*>(sigma_L);
  a.sigR = static_cast<const double2*>(sigma_R);
  a.fL = occupation_L;
  a.fR = occupation_R;
  a.G = static_cast<const double2*>(G);
  a.info = info;
  a.Gless = static_cast<double2*>(G_lesser);
  a.ws = reinterpret_cast<double2*>(static_cast<char*>(workspace) + plan->off_fwd);
  a.ws_chain = plan->ws_chain;
  a.l = (int)d.num_layers;
  a.b = (int)d.block_size;
  a.ne = (int)d.num_energies;
  hipError_t e = d.half_bandwidth == 1
                     ? rgfk::launch_rgf_lesser(a, static_cast<hipStream_t>(stream))
                     : rgfk::launch_nrgf_lesser(a, (int)d.half_bandwidth, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? RGF_OK : RGF_ERR_HIP;
}

rgf_status_t ddrgf_solve(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                         const double* energies, double eta_d, void* G, double* T, int32_t* info,
                         void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return RGF_ERR_INVALID_ARG;
  if (plan->batched || plan->d.method != RGF_METHOD_DDRGF) return RGF_ERR_PLAN_MISMATCH;
  if (!H || !sigma_L || !sigma_R || !energies || !G || !info) return RGF_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < plan->ws_bytes) return RGF_ERR_WORKSPACE_TOO_SMALL;
  const rgf_desc_t& d = plan->d;
  char* ws = static_cast<char*>(workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  TimedScope timed(plan, st);
  const int w = (int)d.half_bandwidth;
  if (plan->ndd) {
    // native n-diagonal DDRGF (separators of w layers)
    const int m = (int)d.num_domains, lr = m * w, wr = 2 * w - 1;
    const size_t bb = (size_t)d.block_size * d.block_size;
    rgfk::NDDArgs a{};
    a.H = static_cast<const double2*>(H);
    a.sigL = static_cast<const double2*>(sigma_L);
    a.sigR = static_cast<const double2*>(sigma_R);
    a.E = energies;
    a.eta_d = eta_d;
    a.G = static_cast<double2*>(G);
    a.T = d.want_transmission ? T : nullptr;
    a.info = info;
    a.l = (int)d.num_layers;
    a.b = (int)d.block_size;
    a.w = w;
    a.m = m;
    a.ne = (int)d.num_energies;
    a.ws_int = reinterpret_cast<double2*>(ws + plan->offn_int);
    a.ws_int_chain = plan->nd_int_chain;
    a.MS = reinterpret_cast<double2*>(ws + plan->offn_ms);
    a.GS = reinterpret_cast<double2*>(ws + plan->offn_gs);
    a.GSlast = reinterpret_cast<double2*>(ws + plan->offn_gslast);
    a.info_part = reinterpret_cast<int*>(ws + plan->offn_info);
    a.info_red = reinterpret_cast<int*>(ws + plan->offn_infored);
    a.ws_fin = reinterpret_cast<double2*>(ws + plan->offn_fin);
    a.herm = reinterpret_cast<int*>(ws + plan->offn_herm);
    rgfk::NSweepArgs r{};
    r.H = a.MS;
    r.direct = 1;
    r.h_stride = (size_t)(2 * wr + 1) * lr * bb;
    r.E = energies;
    r.G = a.GS;
    r.T = nullptr;
    r.info = a.info_red;
    r.ws = reinterpret_cast<double2*>(ws + plan->offn_red);
    r.ws_chain = plan->nd_red_chain;
    r.l = lr;
    r.b = a.b;
    r.w = wr;
    r.ne = a.ne;
    r.nr = w;
    r.rows_last = a.GSlast;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      r.sync = reinterpret_cast<unsigned*>(ws + plan->offn_sync);
      r.spin_limit = DEFAULT_SPLIT_SPIN;
    }
    return rgfk::launch_nddrgf(a, r, st) == hipSuccess ? RGF_OK : RGF_ERR_HIP;
  }
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
  a.herm = reinterpret_cast<int*>(ws + plan->off_herm);
  a.mixed = d.precision == RGF_MIXED_FP32 ? 1 : 0;
  a.kappa_max = kappa_limit(d.mixed_tolerance);
  rgfk::DDArgs a2{};
  double2* band2 = nullptr;
  if (d.inner_domains > 0) {
    // second level: DDRGF on the reduced separator system of every energy
    const int m = a.m, m2 = (int)d.inner_domains;
    const size_t bb = (size_t)a.b * a.b;
    band2 = reinterpret_cast<double2*>(ws + plan->off2_band);
    a2.H = band2;
    a2.direct = 1;
    a2.h_stride = (size_t)3 * m * bb;
    a2.G = a.GS;
    a2.T = nullptr;
    a2.info = a.info_part;
    a2.info_stride = m + 1;
    a2.info_offset = m;
    a2.first_last = a.GSrow + (size_t)(m - 1) * bb;
    a2.first_last_stride = (size_t)m * bb;
    a2.l = m;
    a2.b = a.b;
    a2.m = m2;
    a2.ne = a.ne;
    a2.ws_int = reinterpret_cast<double2*>(ws + plan->off2_int);
    a2.ws_int_chain = plan->dd2_int_chain;
    a2.MS = reinterpret_cast<double2*>(ws + plan->off2_ms);
    a2.GS = reinterpret_cast<double2*>(ws + plan->off2_gs);
    a2.GSrow = reinterpret_cast<double2*>(ws + plan->off2_gsrow);
    a2.ws_red = reinterpret_cast<double2*>(ws + plan->off2_red);
    a2.ws_red_chain = plan->dd2_red_chain;
    a2.ws_fin = reinterpret_cast<double2*>(ws + plan->off2_fin);
    a2.info_part = reinterpret_cast<int*>(ws + plan->off2_info);
    a2.herm = nullptr;
    a2.mixed = 0;
  }
  hipError_t e = rgfk::launch_ddrgf(a, d.inner_domains > 0 ? &a2 : nullptr, band2, st);
  if (e == hipSuccess && w > 1) e = rgfk::launch_unfuse(f, st);
  return e == hipSuccess ? RGF_OK : RGF_ERR_HIP;
}

rgf_status_t rgf_backward(rgf_plan_t plan, const void* H, const void* sigma_L, const void* sigma_R,
                          const double* energies, double eta_d, const void* G_diag, int64_t g_diag_stride,
                          const double* dL_dT, void* dH, double* d_onsite, void* workspace,
                          size_t workspace_bytes, void* stream) {
  if (!plan) return RGF_ERR_INVALID_ARG;
  if (plan->batched || !plan->d.want_backward) return RGF_ERR_PLAN_MISMATCH;
  if (!H || !sigma_L || !sigma_R || !energies || !G_diag || !dL_dT || (!dH && !d_onsite))
    return RGF_ERR_INVALID_ARG;
  if (dH && !(plan->d.want_backward & RGF_BACKWARD_BAND)) return RGF_ERR_PLAN_MISMATCH;
  if (g_diag_stride < 0) return RGF_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < plan->ws_bytes) return RGF_ERR_WORKSPACE_TOO_SMALL;
  TimedScope timed(plan, static_cast<hipStream_t>(stream));
  char* ws = static_cast<char*>(workspace);
  const int l = (int)plan->d.num_layers, b = (int)plan->d.block_size;
  rgfk::AdjArgs a{};
  a.H = static_cast<const double2*>(H);
  a.sigL = static_cast<const double2*>(sigma_L);
  a.sigR = static_cast<const double2*>(sigma_R);
  a.E = energies;
  a.eta_d = eta_d;
  a.Gd = static_cast<const double2*>(G_diag);
  a.gd_stride = g_diag_stride > 0 ? (size_t)g_diag_stride : (size_t)l * b * b;
  a.dLdT = dL_dT;
  a.ck = reinterpret_cast<const double2*>(ws);
  a.ck_chain = plan->ck_chain;
  a.scratch = reinterpret_cast<double2*>(ws + plan->off_adj);
  a.scratch_wg = plan->adj_wg;
  a.gradE = d_onsite ? reinterpret_cast<double*>(ws + plan->off_grad) : nullptr;
  a.hpart = dH ? reinterpret_cast<double2*>(ws + plan->off_hpart) : nullptr;
  a.d_onsite = d_onsite;
  a.dH = static_cast<double2*>(dH);
  a.l = l;
  a.b = b;
  a.ne = (int)plan->d.num_energies;
  a.nd = plan->nd;
  a.dlen = plan->dlen;
  a.nch = plan->nch;
  hipError_t e = rgfk::launch_rgf_adjoint(a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? RGF_OK : RGF_ERR_HIP;
}

rgf_status_t rgf_plan_workspace_bytes(rgf_plan_t plan, size_t* workspace_bytes) {
  if (!plan || !workspace_bytes) return RGF_ERR_INVALID_ARG;
  *workspace_bytes = plan->ws_bytes;
  return RGF_OK;
}

rgf_status_t rgf_lead_workspace_bytes(int64_t block_size, int64_t num_energies, size_t* workspace_bytes) {
  if (!workspace_bytes || block_size < 1 || num_energies < 1) return RGF_ERR_INVALID_ARG;
  if (block_size > 128 || num_energies > (int64_t)1 << 24) return RGF_ERR_UNSUPPORTED;
  const int bp = rgfk::padded_block((int)block_size);
  *workspace_bytes = rgfk::lead_ws_chain_elems(bp) * sizeof(double2) * (size_t)num_energies;
  return RGF_OK;
}

rgf_status_t rgf_lead_self_energy(int64_t block_size, int64_t num_energies, const void* H00, const void* H01,
                                  const void* Hc, const double* energies, double eta, double tolerance,
                                  int32_t max_steps, void* sigma, int32_t* steps, void* workspace,
                                  size_t workspace_bytes, void* stream) {
  size_t need = 0;
  rgf_status_t st = rgf_lead_workspace_bytes(block_size, num_energies, &need);
  if (st != RGF_OK) return st;
  if (!H00 || !H01 || !Hc || !energies || !sigma || !steps) return RGF_ERR_INVALID_ARG;
  if (!(tolerance > 0.0) || max_steps < 1 || !(eta >= 0.0)) return RGF_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < need) return RGF_ERR_WORKSPACE_TOO_SMALL;
  rgfk::LeadArgs a{};
  a.H00 = static_cast<const double2*>(H00);
  a.H01 = static_cast<const double2*>(H01);
  a.Hc = static_cast<const double2*>(Hc);
  a.E = energies;
  a.eta = eta;
  a.tol = tolerance;
  a.max_steps = max_steps;
  a.sigma = static_cast<double2*>(sigma);
  a.steps = steps;
  a.ws = static_cast<double2*>(workspace);
  a.ws_chain = rgfk::lead_ws_chain_elems(rgfk::padded_block((int)block_size));
  a.b = (int)block_size;
  a.ne = (int)num_energies;
  return rgfk::launch_lead_decimation(a, static_cast<hipStream_t>(stream)) == hipSuccess ? RGF_OK : RGF_ERR_HIP;
}

rgf_status_t rgf_plan_set_split(rgf_plan_t plan, int32_t workgroups_per_energy, int64_t spin_limit) {
  if (!plan || spin_limit < 0) return RGF_ERR_INVALID_ARG;
  if (workgroups_per_energy != 0 && workgroups_per_energy != 1 && workgroups_per_energy != 2 &&
      workgroups_per_energy != 4)
    return RGF_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(plan->mu);
  plan->split_want = workgroups_per_energy;
  plan->split_spin = spin_limit;
  plan->split_k = -1;
  return RGF_OK;
}

rgf_status_t rgf_plan_split_workgroups(rgf_plan_t plan, int32_t* workgroups_per_energy) {
  if (!plan || !workgroups_per_energy) return RGF_ERR_INVALID_ARG;
  *workgroups_per_energy = plan->split_used;
  return RGF_OK;
}

rgf_status_t rgf_plan_checkpoint_bytes(rgf_plan_t plan, size_t* checkpoint_bytes) {
  if (!plan || !checkpoint_bytes) return RGF_ERR_INVALID_ARG;
  *checkpoint_bytes = plan->ck_bytes;
  return RGF_OK;
}

rgf_status_t rgf_plan_set_timing(rgf_plan_t plan, int32_t enable, int32_t max_marks) {
  if (!plan) return RGF_ERR_INVALID_ARG;
  for (hipEvent_t ev : plan->tev) hipEventDestroy(ev);
  plan->tev.clear();
  plan->tname.clear();
  plan->tused = plan->tdropped = 0;
  plan->timing = false;
  if (!enable) return RGF_OK;
  if (max_marks < 2) return RGF_ERR_INVALID_ARG;
  try {
    plan->tev.reserve(max_marks);
    plan->tname.assign(max_marks, nullptr);
  } catch (const std::bad_alloc&) {
    return RGF_ERR_OUT_OF_MEMORY;
  }
  for (int i = 0; i < max_marks; ++i) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) {
      for (hipEvent_t x : plan->tev) hipEventDestroy(x);
      plan->tev.clear();
      return RGF_ERR_HIP;
    }
    plan->tev.push_back(ev);
  }
  plan->timing = true;
  return RGF_OK;
}

rgf_status_t rgf_plan_kernel_times(rgf_plan_t plan, rgf_kernel_time_t* out, int32_t max_entries,
                                   int32_t* n_entries, int32_t* dropped) {
  if (!plan || !plan->timing || !out || !n_entries) return RGF_ERR_INVALID_ARG;
  const int used = plan->tused;
  rgf_status_t st = RGF_OK;
  std::vector<const char*> names;
  std::vector<double> ms;
  std::vector<int64_t> cnt;
  if (used > 0 && hipEventSynchronize(plan->tev[used - 1]) != hipSuccess) st = RGF_ERR_HIP;
  for (int i = 1; i < used && st == RGF_OK; ++i) {
    const char* k = plan->tname[i];
    if (!k) continue;   // start mark of the next solve
    float t = 0.f;
    if (hipEventElapsedTime(&t, plan->tev[i - 1], plan->tev[i]) != hipSuccess) {
      st = RGF_ERR_HIP;
      break;
    }
    size_t j = 0;
    while (j < names.size() && std::strcmp(names[j], k) != 0) ++j;
    if (j == names.size()) {
      names.push_back(k);
      ms.push_back(0.0);
      cnt.push_back(0);
    }
    ms[j] += t;
    cnt[j] += 1;
  }
  *n_entries = (int32_t)names.size();
  if (dropped) *dropped = plan->tdropped;
  for (size_t j = 0; j < names.size() && (int)j < max_entries; ++j) {
    std::memset(out[j].name, 0, sizeof out[j].name);
    std::strncpy(out[j].name, names[j], sizeof out[j].name - 1);
    out[j].total_ms = ms[j];
    out[j].launches = cnt[j];
  }
  plan->tused = plan->tdropped = 0;
  return st;
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

int rgf_version(void) { return 200; }


rgf_status_t rgf_dos(const void* G, int64_t num_layers, int64_t block_size, int64_t half_bandwidth,
                     int64_t num_energies, double* dos, void* stream) {
  if (!G || !dos || num_layers < 1 || block_size < 1 || half_bandwidth < 1 || num_energies < 1)
    return RGF_ERR_INVALID_ARG;
  if (num_layers > (int64_t)1 << 24 || block_size > 4096 || num_energies > (int64_t)1 << 24 || half_bandwidth > 64)
    return RGF_ERR_INVALID_ARG;
  return rgfk::launch_dos(static_cast<const double2*>(G), (int)num_layers, (int)block_size, (int)half_bandwidth,
                          (int)num_energies, dos, static_cast<hipStream_t>(stream)) == hipSuccess
             ? RGF_OK
             : RGF_ERR_HIP;
}

rgf_status_t rgf_density(const void* G_lesser, int64_t num_layers, int64_t block_size, int64_t half_bandwidth,
                         int64_t num_energies, const double* weights, double* density, void* stream) {
  if (!G_lesser || !weights || !density || num_layers < 1 || block_size < 1 || half_bandwidth < 1 ||
      num_energies < 1)
    return RGF_ERR_INVALID_ARG;
  if (num_layers > (int64_t)1 << 24 || block_size > 4096 || num_energies > (int64_t)1 << 24 || half_bandwidth > 64)
    return RGF_ERR_INVALID_ARG;
  return rgfk::launch_density(static_cast<const double2*>(G_lesser), (int)num_layers, (int)block_size,
                              (int)half_bandwidth, (int)num_energies, weights, density,
                              static_cast<hipStream_t>(stream)) == hipSuccess
             ? RGF_OK
             : RGF_ERR_HIP;
}

rgf_status_t rgf_bond_current(const void* H, const void* G_lesser, int64_t num_layers, int64_t block_size,
                              int64_t num_energies, double* current, void* stream) {
  if (!H || !G_lesser || !current || num_layers < 2 || block_size < 1 || num_energies < 1)
    return RGF_ERR_INVALID_ARG;
  if (num_layers > (int64_t)1 << 20 || block_size > 4096 || num_energies * (num_layers - 1) > ((int64_t)1 << 31) - 1)
    return RGF_ERR_INVALID_ARG;
  return rgfk::launch_bond_current(static_cast<const double2*>(H), static_cast<const double2*>(G_lesser),
                                   (int)num_layers, (int)block_size, (int)num_energies, current,
                                   static_cast<hipStream_t>(stream)) == hipSuccess
             ? RGF_OK
             : RGF_ERR_HIP;
}

}  // extern "C"
