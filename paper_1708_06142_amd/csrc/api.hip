// C ABI of libocttree: parameter validation, device memory, and the order of
// the solver phases (tree build -> interaction lists -> per-cell evaluation).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "cache.hpp"
#include "ctx.hpp"
#include "kernels.hpp"

using ot::DevBuf;

namespace {

ot_status fail(ot_ctx *c, ot_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

ot_status dev_fail(ot_ctx *c, hipError_t e, const char *what) {
  c->err = std::string(what) + ": " + hipGetErrorString(e);
  return (e == hipErrorOutOfMemory) ? OT_ERR_OOM : OT_ERR_DEVICE;
}

#define HIPCHK(x)                                 \
  do {                                            \
    hipError_t e_ = (x);                          \
    if (e_ != hipSuccess) return dev_fail(c, e_, #x); \
  } while (0)

#define OTCHK(x)                 \
  do {                           \
    ot_status s_ = (x);          \
    if (s_ != OT_OK) return s_;  \
  } while (0)

void release(ot_ctx *c, DevBuf &b) {
  if (b.ptr) {
    (void)hipFree(b.ptr);
    c->dev_bytes -= b.bytes;
  }
  b.ptr = nullptr;
  b.bytes = 0;
}

// Grow-only device allocation accounted against max_device_bytes.
ot_status dalloc(ot_ctx *c, DevBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.ptr && b.bytes >= bytes) return OT_OK;
  release(c, b);
  if (c->p.max_device_bytes && c->dev_bytes + bytes > c->p.max_device_bytes)
    return fail(c, OT_ERR_OOM, "device allocation of " + std::to_string(bytes) +
                                   " bytes exceeds max_device_bytes");
  hipError_t e = hipMalloc(&b.ptr, bytes);
  if (e != hipSuccess) {
    b.ptr = nullptr;
    (void)hipGetLastError();
    return fail(c, e == hipErrorOutOfMemory ? OT_ERR_OOM : OT_ERR_DEVICE,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  b.bytes = bytes;
  c->dev_bytes += bytes;
  return OT_OK;
}

template <typename T>
T *P(DevBuf &b) {
  return static_cast<T *>(b.ptr);
}

ot::DevTree dev_tree(ot_ctx *c) {
  ot::DevTree T;
  T.alev = P<int32_t>(c->alev);
  T.acoord = P<int32_t>(c->acoord);
  T.achild0 = P<int32_t>(c->achild0);
  T.aleaf = P<int32_t>(c->aleaf);
  T.blev = P<int32_t>(c->blev);
  T.bcoord = P<int32_t>(c->bcoord);
  T.bamr = P<int32_t>(c->bamr);
  T.amc = P<double4>(c->amc);
  T.aS = P<double4>(c->aS);
  T.btmc = P<double4>(c->btmc);
  T.cm = P<double>(c->cm);
  T.abq = P<double2>(c->mpe_a);
  T.bbq = P<double2>(c->mpe_b);
  T.na = c->topo.na;
  T.nb = c->topo.nb;
  T.nroots = (int32_t)c->topo.nroots;
  for (int k = 0; k < 3; ++k) {
    T.per[k] = c->p.bc[k];
    T.org[k] = c->p.origin[k];
    T.L[k] = c->box[k];
    T.inv_L[k] = ot::exact_inverse(c->box[k]);
  }
  T.root_size = c->p.root_size;
  return T;
}

template <typename V>
ot_status upload(ot_ctx *c, DevBuf &b, const std::vector<V> &h, hipStream_t st) {
  OTCHK(dalloc(c, b, h.size() * sizeof(V)));
  HIPCHK(hipMemcpyAsync(b.ptr, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, st));
  return OT_OK;
}

ot_status upload_topology(ot_ctx *c, hipStream_t st) {
  const ot::Topology &t = c->topo;
  std::vector<int32_t> child0(t.na), leaf(t.na), bamr(t.nb);
  for (int64_t i = 0; i < t.na; ++i) {
    child0[i] = t.aleaf[i] >= 0 ? -1 : (int32_t)t.achild[8 * i];
    leaf[i] = (int32_t)t.aleaf[i];
  }
  for (int64_t b = 0; b < t.nb; ++b) bamr[b] = (int32_t)t.bamr[b];
  OTCHK(upload(c, c->alev, t.alev, st));
  OTCHK(upload(c, c->acoord, t.acoord, st));
  OTCHK(upload(c, c->achild0, child0, st));
  OTCHK(upload(c, c->aleaf, leaf, st));
  OTCHK(upload(c, c->blev, t.blev, st));
  OTCHK(upload(c, c->bcoord, t.bcoord, st));
  OTCHK(upload(c, c->bamr, bamr, st));
  OTCHK(dalloc(c, c->amc, t.na * sizeof(double4)));
  OTCHK(dalloc(c, c->aS, t.na * sizeof(double4)));
  OTCHK(dalloc(c, c->btmc, t.nb * 72 * sizeof(double4)));
  OTCHK(dalloc(c, c->cm, t.nb * 512 * sizeof(double)));
  OTCHK(dalloc(c, c->flag, 64));
  if (c->p.mac == OT_MAC_MPE) {
    // the leaf blocks under each amr node in depth-first octant order
    std::vector<int32_t> pnode, pblock;
    std::vector<int64_t> poff(t.na + 1, 0);
    std::vector<int64_t> stack;
    for (int64_t i = 0; i < t.na; ++i) {
      poff[i] = (int64_t)pblock.size();
      stack.assign(1, i);
      while (!stack.empty()) {
        const int64_t a = stack.back();
        stack.pop_back();
        if (t.aleaf[a] >= 0) {
          pnode.push_back((int32_t)i);
          pblock.push_back((int32_t)t.aleaf[a]);
        } else {
          for (int o = 7; o >= 0; --o) stack.push_back(t.achild[8 * a + o]);
        }
      }
    }
    poff[t.na] = (int64_t)pblock.size();
    c->mpe_npairs = (int64_t)pblock.size();
    OTCHK(upload(c, c->mpe_pnode, pnode, st));
    OTCHK(upload(c, c->mpe_pblock, pblock, st));
    OTCHK(upload(c, c->mpe_poff, poff, st));
    OTCHK(dalloc(c, c->mpe_part, std::max<int64_t>(c->mpe_npairs, 1) * sizeof(double2)));
    OTCHK(dalloc(c, c->mpe_a, t.na * sizeof(double2)));
    OTCHK(dalloc(c, c->mpe_b, t.nb * 72 * sizeof(double2)));
    HIPCHK(hipStreamSynchronize(st));  // the host vectors end here
  }
  HIPCHK(hipStreamSynchronize(st));
  c->dev_topo = true;
  return OT_OK;
}

ot::EwaldP ewald_desc(const ot_ctx *c) {
  ot::EwaldP E;
  memset(&E, 0, sizeof(E));
  E.bctype = c->bctype;
  E.n = c->ew_n;
  for (int k = 0; k < 3; ++k) {
    E.L[k] = c->box[k];
    E.inv_L[k] = ot::exact_inverse(c->box[k]);
    E.rcp_Lf[k] = (float)(1.0 / c->box[k]);
    E.step[k] = c->ew_step[k];
    E.inv_step[k] = c->ew_step[k] > 0 ? 1.0 / c->ew_step[k] : 0.0;
  }
  if (c->bctype == ot::BC_2P1I) {
    const double Lx = c->box[0], b = c->box[1] / c->box[0];
    const double bL2 = b * Lx * Lx;
    E.zfar = 2.0 * Lx;
    E.far_phi_a = -2.0 * M_PI / bL2;
    E.far_phi_b = std::sqrt(M_PI) / (b * Lx);
    E.far_az = 2.0 * M_PI / bL2;
  }
  if (c->bctype == ot::BC_1P2I) {
    // a line of mass 1/Lx: phi = -(ln(alpha^2 rho^2) + gamma_E)/Lx
    const double Lx = c->box[0], al = c->ew_alpha > 0 ? c->ew_alpha : 2.0 / Lx;
    E.zfar = ot::RFAR_1P2I * Lx;
    E.far_phi_a = -1.0 / Lx;
    E.far_phi_b = -(std::log(al * al) + 0.57721566490153286061) / Lx;
    E.far_az = 2.0 / Lx;
  }
  E.tab64 = static_cast<const double *>(c->tab64.ptr);
  E.tab32 = static_cast<const float4 *>(c->tab32.ptr);
  return E;
}

// Ewald parameters of the context (before any device work)
void ewald_params(ot_ctx *c) {
  const int n = c->p.ewald_n;
  c->ew_n = n;
  c->ew_rcut2 = c->p.ewald_rcut2 > 0 ? c->p.ewald_rcut2 : (c->bctype == ot::BC_3P ? 15 : 10);
  c->ew_fcut2 = c->p.ewald_fcut2 > 0 ? c->p.ewald_fcut2 : 10;
  c->ew_alpha = c->p.ewald_alpha > 0 ? c->p.ewald_alpha : 2.0 / c->box[0];
  c->ew_ext[0] = 0.5 * c->box[0];
  c->ew_ext[1] = 0.5 * c->box[1];
  c->ew_ext[2] = c->bctype == ot::BC_3P ? 0.5 * c->box[2]
                                        : (c->box[2] < 2.0 * c->box[0] ? c->box[2] : 2.0 * c->box[0]);
  if (c->bctype == ot::BC_1P2I) {
    const double rf = ot::RFAR_1P2I * c->box[0];
    c->ew_ext[1] = std::min(c->box[1], rf);
    c->ew_ext[2] = std::min(c->box[2], rf);
  }
  for (int k = 0; k < 3; ++k) c->ew_step[k] = c->ew_ext[k] / (double)(n - 1);
}

// every input the table depends on
ot::CacheKey ewald_key(const ot_ctx *c) {
  ot::CacheKey k;
  memset(&k, 0, sizeof(k));
  k.kind = 1;
  k.i[0] = c->bctype;
  k.i[1] = c->ew_n;
  k.i[2] = c->ew_rcut2;
  k.i[3] = c->ew_fcut2;
  k.i[4] = 10;  // channels per point, x fastest, FP64
  k.d[0] = c->ew_alpha;
  for (int q = 0; q < 3; ++q) {
    k.d[1 + q] = c->box[q];
    k.d[4 + q] = c->ew_ext[q];
  }
  return k;
}

ot_status ewald_prepare(ot_ctx *c, const char *cache, hipStream_t st) {
  if (c->bctype == ot::BC_ISO) return fail(c, OT_ERR_STATE, "Ewald table needs periodic or mixed boundaries");
  std::string why;
  if (cache && !ot::cache_path_usable(cache, why)) return fail(c, OT_ERR_IO, why);
  if (!c->ewald_ready) ewald_params(c);
  const size_t np = (size_t)c->ew_n * c->ew_n * c->ew_n;
  const ot::CacheKey key = ewald_key(c);
  std::vector<char> payload;
  ot::CacheRead cr = ot::CacheRead::Regenerate;
  if (cache) {
    cr = ot::cache_read(cache, key, payload, why);
    if (cr == ot::CacheRead::IoError) return fail(c, OT_ERR_IO, why);
    if (cr == ot::CacheRead::Loaded && payload.size() != np * 10 * sizeof(double)) cr = ot::CacheRead::Regenerate;
  }
  if (c->ewald_ready && !cache) return OT_OK;
  HIPCHK(hipSetDevice(c->p.device));
  if (!c->ewald_ready) {
    OTCHK(dalloc(c, c->tab64, np * 10 * sizeof(double)));
    OTCHK(dalloc(c, c->tab32, np * 3 * sizeof(float4)));
    ot::EwaldP E = ewald_desc(c);
    if (cr == ot::CacheRead::Loaded) {
      HIPCHK(hipMemcpyAsync(c->tab64.ptr, payload.data(), payload.size(), hipMemcpyHostToDevice, st));
      HIPCHK(ot::launch_ewald_pack32(E, P<double>(c->tab64), P<float4>(c->tab32), st));
    } else {
      HIPCHK(ot::launch_ewald_table(E, c->ew_alpha, c->ew_rcut2, c->ew_fcut2, P<double>(c->tab64),
                                    P<float4>(c->tab32), st));
    }
    HIPCHK(hipStreamSynchronize(st));
    c->ewald_ready = true;
  }
  if (cache && cr != ot::CacheRead::Loaded) {
    std::vector<double> h(np * 10);
    HIPCHK(hipMemcpy(h.data(), c->tab64.ptr, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (!ot::cache_write(cache, key, h.data(), h.size() * sizeof(double), why)) return fail(c, OT_ERR_IO, why);
  }
  return OT_OK;
}

int npix_of(const ot_ctx *c) { return 12 * c->p.nside * c->p.nside; }

ot::RayTableP raytable_desc(const ot_ctx *c) {
  ot::RayTableP P;
  P.nside = c->p.nside;
  P.npix = npix_of(c);
  P.ntheta = c->p.il_ntheta;
  P.nphi = c->p.il_nphi;
  P.npsi = c->p.il_npsi;
  P.nr = c->p.il_nr;
  P.nazi = c->p.il_nazi;
  P.nentries = (int64_t)P.ntheta * P.nphi * P.npsi;
  P.dtheta = M_PI / (double)P.ntheta;
  P.dphi = (2.0 * M_PI) / (double)P.nphi;
  P.dpsi = c->p.psi_max / (double)P.npsi;
  return P;
}

// Direction-bin look-up tables of the column walk.  Each angle's bin edges
// are mapped to a variable that increases or decreases with the angle: cos
// theta on [-1, 1] for theta, sin psi on [0, 1] for psi (edges above pi/2 are
// never reached), t = cos phi / (|cos phi| + sin phi) on [-1, 1] for phi in
// [0, pi] (bins below half).  The cells are at most half as wide as the
// closest two edges; a cell holds the lowest bin over the cell widened by
// LUT_GUARD on both sides (far more than the FP32 rounding of the variable and
// of the cell index), so a widened cell spans at most one edge and the bin of
// any value mapped to the cell is its entry or one more.
constexpr double LUT_GUARD = 1e-5;

struct BinLut {
  int m[3];  // cells: theta, psi, phi
  bool ok;   // every table fits its share of LUT_BYTES
};

std::vector<double> lut_edges(const ot::RayTableP &RP, int which) {
  std::vector<double> x;
  if (which == 0)
    for (int k = 1; k < RP.ntheta; ++k) x.push_back(std::cos(k * RP.dtheta));
  else if (which == 1)
    for (int k = 1; k < RP.npsi && k * RP.dpsi <= 0.5 * M_PI; ++k) x.push_back(std::sin(k * RP.dpsi));
  else
    for (int q = 1; q < RP.nphi / 2; ++q) {
      const double cq = std::cos(q * RP.dphi), sq = std::sin(q * RP.dphi);
      x.push_back(cq / (std::fabs(cq) + sq));
    }
  return x;
}

BinLut bin_lut_plan(const ot::RayTableP &RP) {
  BinLut L;
  const double range[3] = {2.0, 1.0, 2.0};
  const int cap[3] = {ot::LUT_TH, ot::LUT_PS, ot::LUT_PH};
  L.ok = true;
  for (int w = 0; w < 3; ++w) {
    const std::vector<double> x = lut_edges(RP, w);
    double gap = HUGE_VAL;
    for (size_t i = 1; i < x.size(); ++i) gap = std::min(gap, std::fabs(x[i] - x[i - 1]));
    const double cells = gap == HUGE_VAL ? 2.0 : std::ceil(range[w] / (0.5 * gap));
    const bool fits = cells + 1 <= cap[w] && (gap == HUGE_VAL || gap > 100.0 * LUT_GUARD);
    L.m[w] = fits ? (int)cells : 1;
    L.ok = L.ok && fits;
  }
  return L;
}

std::vector<uint8_t> bin_luts(const ot::RayTableP &RP) {
  const BinLut L = bin_lut_plan(RP);
  std::vector<uint8_t> lut(ot::LUT_BYTES, 0);
  if (!L.ok) return lut;
  const int base[3] = {0, ot::LUT_TH, ot::LUT_TH + ot::LUT_PS};
  const double lo0[3] = {-1.0, 0.0, -1.0}, range[3] = {2.0, 1.0, 2.0};
  for (int w = 0; w < 3; ++w) {
    const std::vector<double> x = lut_edges(RP, w);
    const double width = range[w] / L.m[w];
    for (int j = 0; j <= L.m[w]; ++j) {
      // theta and phi bins grow as their variable falls (lowest bin at the
      // widened cell's top), the psi bin as sin psi rises (at its bottom)
      const double v = w == 1 ? lo0[w] + j * width - LUT_GUARD : lo0[w] + (j + 1) * width + LUT_GUARD;
      int bin = 0;
      for (double xe : x) bin += w == 1 ? v >= xe : v <= xe;
      lut[base[w] + j] = (uint8_t)bin;
    }
  }
  return lut;
}

// Half-width of the lattice table (cells of a block's own size within LAT_R
// cell sizes per axis): the walk takes a record to the table when all 512
// cells of the block see it within the table, i.e. from LAT_R - 7 cells before
// the block's first cell to LAT_R cells after it.  In the lists of a 128^3
// lognormal field under APE every cell of the block's own size lies inside.
// 47^3 rows of 68 bytes (head, four-slot record, FP64 weights).
constexpr int LAT_R = 23;

ot::ColP col_params(ot_ctx *c);

ot_status raytable_prepare(ot_ctx *c, hipStream_t st) {
  if (c->p.nside <= 0) return fail(c, OT_ERR_STATE, "columns are off (nside = 0)");
  if (c->rt_ready) return OT_OK;
  HIPCHK(hipSetDevice(c->p.device));
  const ot::RayTableP RP = raytable_desc(c);
  DevBuf dense, cnt;
  ot_status s = dalloc(c, dense, (size_t)RP.nentries * RP.npix * sizeof(double));
  if (s == OT_OK) s = dalloc(c, cnt, (size_t)RP.nentries * sizeof(int32_t));
  if (s == OT_OK) s = dalloc(c, c->rt_off, (size_t)(RP.nentries + 1) * sizeof(int64_t));
  int64_t total = 0;
  hipError_t e = hipSuccess;
  if (s == OT_OK)
    e = ot::launch_raytable(RP, P<double>(dense), P<int32_t>(cnt), P<int64_t>(c->rt_off), nullptr, nullptr,
                            &total, st);
  if (s == OT_OK && e == hipSuccess) {
    s = dalloc(c, c->rt_pix, (size_t)total * sizeof(uint16_t));
    if (s == OT_OK) s = dalloc(c, c->rt_w64, (size_t)total * sizeof(double));
    // the rows of the cells at lattice offsets follow the table's own rows
    const int64_t nlat = (2 * LAT_R + 1) * (2 * LAT_R + 1) * (2 * LAT_R + 1);
    if (s == OT_OK) s = dalloc(c, c->rt_rows, (size_t)(RP.nentries + nlat) * sizeof(uint32_t));
    if (s == OT_OK) s = dalloc(c, c->rt_ent, (size_t)total * sizeof(uint32_t));
    if (s == OT_OK) s = dalloc(c, c->rt_rows8, (size_t)(RP.nentries + nlat) * 32);
    if (s == OT_OK) s = dalloc(c, c->rt_quad64, (size_t)(RP.nentries + nlat) * 32);
    if (s == OT_OK) s = dalloc(c, c->rt_lut, ot::LUT_BYTES);
    if (s == OT_OK && total >= ((int64_t)1 << 26)) s = fail(c, OT_ERR_UNSUPPORTED, "node-ray table too large");
    if (s == OT_OK) {
      // packed rows hold at most 63 pixels per entry
      std::vector<int64_t> offh(RP.nentries + 1);
      e = hipMemcpy(offh.data(), c->rt_off.ptr, offh.size() * sizeof(int64_t), hipMemcpyDeviceToHost);
      for (int64_t q = 0; e == hipSuccess && s == OT_OK && q < RP.nentries; ++q)
        if (offh[q + 1] - offh[q] > 63) s = fail(c, OT_ERR_UNSUPPORTED, "node-ray table row with > 63 pixels");
    }
    if (s == OT_OK) {
      // the sizing pass is repeated (deterministic) and the rows are filled
      e = ot::launch_raytable(RP, P<double>(dense), P<int32_t>(cnt), P<int64_t>(c->rt_off),
                              P<uint16_t>(c->rt_pix), P<double>(c->rt_w64), &total, st);
      if (e == hipSuccess)
        e = ot::launch_raytable_pack(RP, P<int64_t>(c->rt_off), P<uint16_t>(c->rt_pix), P<double>(c->rt_w64),
                                     P<uint32_t>(c->rt_rows), P<uint32_t>(c->rt_ent), P<uint4>(c->rt_rows8),
                                     P<double>(c->rt_quad64), st);
      // direction-bin thresholds: c |c| with c = cos(k dtheta), sin^2(k dpsi),
      // (cos(k dphi), sin(k dphi)) pairs; each list ends in a threshold its test
      // never passes (-inf, +inf, and phi = pi exactly as cos -1, sin 0)
      std::vector<double> thr;
      for (int k = 0; k < RP.ntheta; ++k) {
        const double c = std::cos(k * RP.dtheta);
        thr.push_back(c * std::fabs(c));
      }
      thr.push_back(-HUGE_VAL);
      for (int k = 0; k < RP.npsi; ++k) {
        // psi <= pi/2: a bin edge above it is never reached
        const double sn = std::sin(k * RP.dpsi);
        thr.push_back(k * RP.dpsi > 0.5 * M_PI ? HUGE_VAL : sn * sn);
      }
      thr.push_back(HUGE_VAL);
      const int half = RP.nphi / 2;
      for (int k = 0; k <= half; ++k) {
        thr.push_back(k == half ? -1.0 : std::cos(k * RP.dphi));
        thr.push_back(k == half ? 0.0 : std::sin(k * RP.dphi));
      }
      if (e == hipSuccess && (s = dalloc(c, c->rt_thr, thr.size() * sizeof(double))) == OT_OK)
        e = hipMemcpyAsync(c->rt_thr.ptr, thr.data(), thr.size() * sizeof(double), hipMemcpyHostToDevice, st);
      const std::vector<uint8_t> lut = bin_luts(RP);
      if (e == hipSuccess && s == OT_OK)
        e = hipMemcpyAsync(c->rt_lut.ptr, lut.data(), lut.size(), hipMemcpyHostToDevice, st);
      // rows of the cells at lattice offsets, by the walk's own binning
      if (e == hipSuccess && s == OT_OK)
        e = ot::launch_lattice_rows(col_params(c), LAT_R, P<uint32_t>(c->rt_rows), P<uint4>(c->rt_rows8),
                                    P<double>(c->rt_quad64), st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
  }
  release(c, dense);
  release(c, cnt);
  if (s != OT_OK) return s;
  if (e != hipSuccess) return dev_fail(c, e, "node-ray table");
  c->rt_pairs = total;
  c->rt_ready = true;
  return OT_OK;
}

// Every cell centre org + (i + 1/2) h is an exact double: the root size is a
// power of two and the origin a multiple of half the finest cell size, within
// 2^40 of them (so same-size cells lie exact multiples of h apart).
bool dyadic_grid(const ot_ctx *c) {
  if (!c->have_blocks) return false;
  int ex = 0;
  if (!(c->p.root_size > 0) || std::frexp(c->p.root_size, &ex) != 0.5) return false;
  const double half = ot::size_at(c->p.root_size, c->topo.lmax) / 16.0;
  for (int k = 0; k < 3; ++k) {
    const double q = c->p.origin[k] / half;
    if (q != std::floor(q) || std::fabs(q) > 0x1p40 || q * half != c->p.origin[k]) return false;
    if ((double)c->p.nroot[k] * c->p.root_size / half > 0x1p40) return false;
  }
  return true;
}

ot::ColP col_params(ot_ctx *c) {
  ot::ColP C;
  const ot::RayTableP RP = raytable_desc(c);
  C.npix = RP.npix;
  C.ntheta = RP.ntheta;
  C.nphi = RP.nphi;
  C.npsi = RP.npsi;
  C.dtheta = RP.dtheta;
  C.dphi = RP.dphi;
  C.dpsi = RP.dpsi;
  C.req = 0.6203504908994001;  // (3 / (4 pi))^(1/3)
  C.omega = 4.0 * M_PI / (double)RP.npix;
  C.kappa = c->p.kappa;
  C.max_dist2 = c->p.max_dist * c->p.max_dist;
  C.ip_pi = std::min((int)std::floor(M_PI / RP.dphi), RP.nphi - 1);
  C.nthr = (RP.ntheta + 1) + (RP.npsi + 1) + 2 * (RP.nphi / 2 + 1);
  const BinLut L = bin_lut_plan(RP);
  C.estimate = L.ok;
  C.lut_th = (float)(0.5 * L.m[0]);
  C.lut_ps = (float)L.m[1];
  C.lut_ph = (float)(0.5 * L.m[2]);
  C.thr = P<double>(c->rt_thr);
  C.lut = P<uint8_t>(c->rt_lut);
  C.rows = P<uint32_t>(c->rt_rows);
  C.rows8 = P<uint4>(c->rt_rows8);
  C.quad_w64 = P<double>(c->rt_quad64);
  C.lat0 = (int)RP.nentries;
  C.lat_r = c->rt_ready && dyadic_grid(c) ? LAT_R : 0;
  C.pix = P<uint16_t>(c->rt_pix);
  C.w64 = P<double>(c->rt_w64);
  C.ent = P<uint32_t>(c->rt_ent);
  return C;
}

// Interaction lists for the given MAC: count, scan, fill.
ot_status build_lists(ot_ctx *c, const ot::MacP &mp, bool sizes, hipStream_t st, int sub = 0) {
  // the host's copy of the offsets describes the previous lists until the
  // caller refreshes it: exports wait for that
  c->lists_valid = false;
  const ot::Topology &t = c->topo;
  ot::DevTree T = dev_tree(c);
  const int64_t ntg = sub ? 8 * t.nb : t.nb;
  int64_t capA = 0;
  for (int l = 1; l <= t.lmax; ++l) capA = std::max(capA, t.level_begin[l + 1] - t.level_begin[l]);
  const int64_t stride = 2 * capA + 9 * t.nb;
  int64_t grid = std::min<int64_t>(ntg, 2048);
  const int64_t budget = (int64_t)1 << 30;  // scratch bytes
  while (grid > 64 && grid * stride * 4 > budget) grid /= 2;
  OTCHK(dalloc(c, c->lscratch, (size_t)(grid * stride * 4)));
  OTCHK(dalloc(c, c->lcount, ntg * sizeof(int32_t)));
  OTCHK(dalloc(c, c->loff, (ntg + 1) * sizeof(int64_t)));
  OTCHK(dalloc(c, c->lnodes, 2 * ntg * sizeof(int32_t)));
  HIPCHK(ot::launch_lists(false, T, mp, (int)grid, P<int32_t>(c->lcount), P<int32_t>(c->lnodes), nullptr, nullptr, nullptr,
                          nullptr, P<int32_t>(c->lscratch), stride, capA, st, nullptr, 0, sub));
  HIPCHK(ot::launch_scan(P<int32_t>(c->lcount), ntg, P<int64_t>(c->loff), st));
  int64_t total = 0;
  HIPCHK(hipMemcpyAsync(&total, P<int64_t>(c->loff) + ntg, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  OTCHK(dalloc(c, c->lrec, (size_t)total * sizeof(double4)));
  OTCHK(dalloc(c, c->lid, (size_t)total * sizeof(int32_t)));
  if (sizes) OTCHK(dalloc(c, c->lh, (size_t)total * sizeof(double)));
  HIPCHK(ot::launch_lists(true, T, mp, (int)grid, P<int32_t>(c->lcount), nullptr, P<int64_t>(c->loff),
                          P<double4>(c->lrec), P<int32_t>(c->lid), sizes ? P<double>(c->lh) : nullptr,
                          P<int32_t>(c->lscratch), stride, capA, st, nullptr, 0, sub));
  c->list_cap = total;
  c->list_sub = sub;
  return OT_OK;
}

ot::MacP mac_params(const ot_ctx *c, int mac, double a_lim, bool cols) {
  ot::MacP m;
  m.theta2 = c->p.theta_lim * c->p.theta_lim;
  m.half_eta = 0.5 * c->p.eta_sb;
  m.G = c->p.G;
  m.a_lim = a_lim;
  const double tp = c->p.theta_pix > 0 ? c->p.theta_pix : 1.0 / (double)(c->p.nside > 0 ? c->p.nside : 1);
  m.tpix2 = tp * tp;
  m.mac = mac;
  m.use_pix = cols ? 1 : 0;
  return m;
}

// a_lim = eps_lim * max |a| from a BH FP64 walk (Sec. 3)
ot_status ape_limit(ot_ctx *c, hipStream_t st, double *alim) {
  if (c->p.a_lim > 0) {
    *alim = c->p.a_lim;
    return OT_OK;
  }
  if (!c->alim_valid) {
    OTCHK(build_lists(c, mac_params(c, OT_MAC_BH, 0.0, false), false, st));
    const int64_t ncell = c->topo.nb * 512;
    DevBuf phi, acc, mx;
    OTCHK(dalloc(c, phi, ncell * sizeof(double)));
    ot_status s = dalloc(c, acc, 3 * ncell * sizeof(double));
    if (s == OT_OK) s = dalloc(c, mx, sizeof(unsigned long long));
    unsigned long long bits = 0;
    hipError_t e = hipSuccess;
    if (s == OT_OK) {
      ot::DevTree T = dev_tree(c);
      e = hipMemsetAsync(mx.ptr, 0, sizeof(unsigned long long), st);
      if (e == hipSuccess)
        e = ot::launch_eval64(T, ewald_desc(c), P<int64_t>(c->loff), P<double4>(c->lrec),
                              P<double>(phi), P<double>(acc), c->p.G, st);
      if (e == hipSuccess) e = ot::launch_amax(P<double>(acc), ncell, P<unsigned long long>(mx), st);
      if (e == hipSuccess) e = hipMemcpyAsync(&bits, mx.ptr, sizeof(bits), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    release(c, phi);
    release(c, acc);
    release(c, mx);
    if (s != OT_OK) return s;
    if (e != hipSuccess) return dev_fail(c, e, "a_max pre-pass");
    double a2;
    memcpy(&a2, &bits, sizeof(double));
    c->alim = c->p.eps_lim * std::sqrt(a2);
    c->alim_valid = true;
  }
  *alim = c->alim;
  return OT_OK;
}

// ---------------------------------------------------------------- surrogate
// A device buffer released when it goes out of scope (training scratch).
struct Scoped {
  ot_ctx *c;
  DevBuf b;
  explicit Scoped(ot_ctx *cc) : c(cc) {}
  ~Scoped() { release(c, b); }
  template <typename T>
  T *p() { return static_cast<T *>(b.ptr); }
};

ot::MlpNorm mlp_norm_of(const ot_ctx *c) {
  using ot::mlpdef::NO;
  ot::MlpNorm N;
  for (int k = 0; k < 3; ++k) N.ext[k] = c->mlp_norm[k];
  for (int o = 0; o < NO; ++o) {
    N.mu[o] = c->mlp_norm[3 + o];
    N.sig[o] = c->mlp_norm[3 + NO + o];
  }
  return N;
}

// Largest Taylor offset per axis the surrogate walk allows (half the Ewald
// table's smallest spacing) and the grid's largest cell size.
double mlp_tmax(const ot_ctx *c) {
  const double reach = c->p.mlp_reach > 0.0 ? c->p.mlp_reach : 1.0;
  return reach * (0.5 * std::min(c->ew_step[0], std::min(c->ew_step[1], c->ew_step[2])));
}
double cell_size_max(const ot_ctx *c) {
  int lmin = c->topo.lmax;
  for (int32_t l : c->topo.blev) lmin = std::min(lmin, (int)l);
  return ot::size_at(c->p.root_size, lmin) / 8.0;
}

// pack the current parameters into the inference operands
ot_status mlp_pack(ot_ctx *c, hipStream_t st) {
  OTCHK(dalloc(c, c->mlp_pk, (size_t)ot::mlpdef::NPK * 64 * 16));
  HIPCHK(ot::launch_mlp_pack(P<float>(c->mlp_P), mlp_norm_of(c), c->mlp_pk.ptr, st));
  return OT_OK;
}

// correction at n device offsets by one method into out [n][10]
ot_status ewald_points(ot_ctx *c, int method, int64_t n, const double *d, double *out, hipStream_t st) {
  const ot::EwaldP E = ewald_desc(c);
  if (method == OT_EWALD_MLP) {
    if (!c->mlp_have) return fail(c, OT_ERR_STATE, "no surrogate installed");
    HIPCHK(ot::launch_mlp_points_eval(c->mlp_pk.ptr, E, n, d, out, st));
  } else {
    HIPCHK(ot::launch_ewald_points10(method == OT_EWALD_EXACT ? 1 : 0, E, c->ew_alpha, c->ew_rcut2, c->ew_fcut2,
                                     n, d, out, st));
  }
  return OT_OK;
}

ot_status mlp_grad_scratch(ot_ctx *c, int64_t batch) {
  const int64_t np = ot::mlp_partials(batch);
  OTCHK(dalloc(c, c->mlp_part, (size_t)np * ot::mlpdef::NP * sizeof(float)));
  OTCHK(dalloc(c, c->mlp_lossp, (size_t)np * sizeof(float)));
  return OT_OK;
}

// list lengths, their histogram and the MAC suite's opened / accepted counts
// (nodes: per block the opened nodes and the cells of its list, or empty)
void list_stats(const ot_ctx *c, const std::vector<int32_t> &nodes, ot_stats *stats) {
  memset(stats, 0, sizeof(*stats));
  int64_t mx = 0;
  const int64_t ntg = c->list_sub ? 8 * c->topo.nb : c->topo.nb;
  for (int64_t b = 0; b < ntg; ++b) {
    const int64_t len = c->off_host[b + 1] - c->off_host[b];
    mx = std::max(mx, len);
    int k = 0;
    while (k < 31 && ((int64_t)2 << k) <= len) ++k;
    ++stats->list_hist[k];
    if (!nodes.empty()) {
      stats->n_opened += nodes[2 * b];
      stats->n_accepted += len - nodes[2 * b + 1];
    }
  }
  stats->total_list = c->off_host[ntg];
  stats->max_list = mx;
  stats->n_interactions = (c->list_sub ? 64 : 512) * (stats->total_list - ntg);
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.f;
  return ms;
}

ot_status solve_impl(ot_ctx *c, bool fp64, void *phi, void *acc, void *npix, void *tau, ot_stats *stats,
                     void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (!phi || !acc) return fail(c, OT_ERR_INVALID_ARG, "phi and acc must be device pointers");
  const bool cols = c->p.nside > 0;
  if (cols && (!npix || !tau)) return fail(c, OT_ERR_INVALID_ARG, "nside > 0 needs npix and tau outputs");
  if (!c->built) return fail(c, OT_ERR_STATE, "ot_solve before a successful ot_build");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->p.device));
  if (c->bctype != ot::BC_ISO) {
    if (c->p.ewald == OT_EWALD_EXACT)
      return fail(c, OT_ERR_UNSUPPORTED, "per-pair exact Ewald series is not built into the walk");
    OTCHK(ewald_prepare(c, nullptr, st));
  }
  const bool use_mlp = (c->bctype == ot::BC_3P || c->bctype == ot::BC_2P1I) && c->p.ewald == OT_EWALD_MLP &&
                       c->mlp_ok && !fp64;
  if (cols) OTCHK(raytable_prepare(c, st));
  double alim = 0.0;
  if (c->p.mac == OT_MAC_APE || c->p.mac == OT_MAC_MPE) OTCHK(ape_limit(c, st, &alim));
  for (int i = 0; i < 6; ++i)
    if (!c->ev[i]) HIPCHK(hipEventCreate(&c->ev[i]));
  // with the surrogate and maps too large for LDS, one kernel carries both
  // the surrogate's gravity and the columns
  const bool fused = use_mlp && cols && ot::cols_lds_cpw(npix_of(c), false, col_params(c).nthr) == 0;
  // one list per 4^3 block octant: only this kernel walks them, and its
  // octants hold whole cell groups of 2^3 or 4^3 cells
  const int sub = c->p.list_group == 4 ? 1 : 0;
  if (sub && !(fused && ot::mlp_group_level(cell_size_max(c), mlp_tmax(c)) >= 1))
    return fail(c, OT_ERR_UNSUPPORTED,
                "list_group 4 needs the FP32 walk with an accepted surrogate (3P or 2P1I), Nside 4 columns and "
                "cell groups of 2^3 or more cells");
  HIPCHK(hipEventRecord(c->ev[0], st));
  OTCHK(build_lists(c, mac_params(c, c->p.mac, alim, cols), cols, st, sub));
  HIPCHK(hipEventRecord(c->ev[1], st));
  ot::DevTree T = dev_tree(c);
  ot::EwaldP E = ewald_desc(c);
  int wg_per_cu = 0;
  if (fused) OTCHK(dalloc(c, c->llat, (size_t)c->list_cap * sizeof(int32_t)));
  if (use_mlp && !fused)
    // gravity from the surrogate walk (the columns, if any, follow without gravity)
    HIPCHK(ot::launch_eval_mlp(T, E, c->mlp_pk.ptr, P<int64_t>(c->loff), P<double4>(c->lrec), (float *)phi,
                               (float *)acc, c->p.G, mlp_tmax(c), cell_size_max(c), st));
  HIPCHK(hipEventRecord(c->ev[4], st));
  if (fused) {
    HIPCHK(ot::launch_eval_cols_mlp(T, E, col_params(c), c->mlp_pk.ptr, P<int64_t>(c->loff), P<double4>(c->lrec),
                                    P<int32_t>(c->lid), P<double>(c->lh), P<int32_t>(c->llat), (float *)phi,
                                    (float *)acc, (float *)npix, (float *)tau,
                                    c->p.G, mlp_tmax(c), cell_size_max(c), &wg_per_cu, st, sub));
  } else if (cols) {
    // maps in LDS when 128 or more cells' maps fit there, else in npix
    const ot::ColP C = col_params(c);
    HIPCHK(ot::launch_eval_cols(fp64, T, E, C, P<int64_t>(c->loff), P<double4>(c->lrec), P<int32_t>(c->lid),
                                P<double>(c->lh), phi, acc, npix, tau, c->p.G,
                                ot::cols_lds_cpw(C.npix, fp64, C.nthr), use_mlp, &wg_per_cu, st));
  } else if (fp64)
    HIPCHK(ot::launch_eval64(T, E, P<int64_t>(c->loff), P<double4>(c->lrec), (double *)phi,
                             (double *)acc, c->p.G, st));
  else if (use_mlp) {
  } else
    HIPCHK(ot::launch_eval32(T, E, P<int64_t>(c->loff), P<double4>(c->lrec), P<int32_t>(c->lid),
                             (float *)phi, (float *)acc, c->p.G, st));
  HIPCHK(hipEventRecord(c->ev[2], st));
  const int64_t ntg = sub ? 8 * c->topo.nb : c->topo.nb;
  c->off_host.resize(ntg + 1);
  HIPCHK(hipMemcpyAsync(c->off_host.data(), c->loff.ptr, (ntg + 1) * sizeof(int64_t),
                        hipMemcpyDeviceToHost, st));
  std::vector<int32_t> nodes;
  if (stats) {
    nodes.resize(2 * ntg);
    HIPCHK(hipMemcpyAsync(nodes.data(), c->lnodes.ptr, nodes.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                          st));
  }
  HIPCHK(hipStreamSynchronize(st));
  c->lists_valid = true;
  if (stats) {
    list_stats(c, nodes, stats);
    stats->a_lim_used = alim;
    stats->ms_list = elapsed(c->ev[0], c->ev[1]);
    stats->ms_eval = elapsed(c->ev[1], c->ev[2]);
    stats->ms_build = c->ms_build;
    stats->ewald_used = use_mlp ? OT_EWALD_MLP : OT_EWALD_TABLE;
    stats->eval_wg_per_cu = wg_per_cu;
    if (use_mlp) {
      stats->ms_gravity = fused ? 0.0 : elapsed(c->ev[1], c->ev[4]);
      const double tmax = mlp_tmax(c);
      for (int64_t q = 0; q < ntg; ++q) {
        const int64_t b = sub ? q >> 3 : q;
        stats->n_mlp_evals += (int64_t)ot::mlp_groups(ot::size_at(c->p.root_size, c->topo.blev[b]) / 8.0, tmax) /
                              (sub ? 8 : 1) * (c->off_host[q + 1] - c->off_host[q]);
      }
    }
    if (cols) stats->ms_columns = elapsed(c->ev[4], c->ev[2]);
  }
  return OT_OK;
}

// Adaptive block update (Sec. 2.2.6): the eight corner cells of every block
// first (FP64 gravity, against the previous acceleration in acc), then the
// full evaluation (with the columns when nside > 0) of the blocks where one of
// them moved by tol or more; the other blocks keep phi, acc, npix and tau.
ot_status abu_impl(ot_ctx *c, bool fp64, void *phi, void *acc, void *npix, void *tau, double tol,
                   double tol_tau, int32_t *updated, ot_stats *stats, void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (!phi || !acc) return fail(c, OT_ERR_INVALID_ARG, "phi and acc must be device pointers");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(c, OT_ERR_INVALID_ARG, "tol must be finite and >= 0");
  const bool cols = c->p.nside > 0;
  if (cols && (!npix || !tau)) return fail(c, OT_ERR_INVALID_ARG, "nside > 0 needs npix and tau");
  if (cols && (!(tol_tau >= 0.0) || !std::isfinite(tol_tau)))
    return fail(c, OT_ERR_INVALID_ARG, "tol_tau must be finite and >= 0");
  if (!c->built) return fail(c, OT_ERR_STATE, "ot_solve_abu before a successful ot_build");
  if (c->p.list_group == 4) return fail(c, OT_ERR_UNSUPPORTED, "the adaptive update walks one list per block");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->p.device));
  if (c->bctype != ot::BC_ISO) {
    if (c->p.ewald == OT_EWALD_EXACT)
      return fail(c, OT_ERR_UNSUPPORTED, "per-pair exact Ewald series is not built into the walk");
    if (c->p.ewald == OT_EWALD_MLP && !fp64)
      return fail(c, OT_ERR_UNSUPPORTED, "the adaptive block update uses the Ewald table");
    OTCHK(ewald_prepare(c, nullptr, st));
  }
  if (cols) OTCHK(raytable_prepare(c, st));
  double alim = 0.0;
  if (c->p.mac == OT_MAC_APE || c->p.mac == OT_MAC_MPE) OTCHK(ape_limit(c, st, &alim));
  for (int i = 0; i < 4; ++i)
    if (!c->ev[i]) HIPCHK(hipEventCreate(&c->ev[i]));
  const int64_t nb = c->topo.nb;
  // grow-only: a later ot_set_blocks may have brought more blocks
  OTCHK(dalloc(c, c->abu_flag, nb * sizeof(int32_t)));
  OTCHK(dalloc(c, c->abu_blist, nb * sizeof(int32_t)));
  if (c->abu_flag.bytes < (size_t)nb * sizeof(int32_t) || c->abu_blist.bytes < (size_t)nb * sizeof(int32_t))
    return fail(c, OT_ERR_STATE, "adaptive block update buffers smaller than the block count");
  HIPCHK(hipEventRecord(c->ev[0], st));
  OTCHK(build_lists(c, mac_params(c, c->p.mac, alim, cols), cols, st));
  HIPCHK(hipEventRecord(c->ev[1], st));
  ot::DevTree T = dev_tree(c);
  ot::EwaldP E = ewald_desc(c);
  HIPCHK(hipMemsetAsync(c->abu_flag.ptr, 0, nb * sizeof(int32_t), st));
  HIPCHK(ot::launch_abu_corners(fp64, T, E, P<int64_t>(c->loff), P<double4>(c->lrec), acc, c->p.G, tol,
                                P<int32_t>(c->abu_flag), st));
  if (cols)
    HIPCHK(ot::launch_abu_corner_cols(fp64, T, E, col_params(c), P<int64_t>(c->loff), P<double4>(c->lrec),
                                      P<double>(c->lh), npix, tol_tau, P<int32_t>(c->abu_flag), st));
  std::vector<int32_t> flag(nb), blist;
  HIPCHK(hipMemcpyAsync(flag.data(), c->abu_flag.ptr, nb * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int64_t b = 0; b < nb; ++b)
    if (flag[b]) blist.push_back((int32_t)b);
  if (updated) memcpy(updated, flag.data(), nb * sizeof(int32_t));
  const int64_t nup = (int64_t)blist.size();
  if (nup > 0)
    HIPCHK(hipMemcpyAsync(c->abu_blist.ptr, blist.data(), nup * sizeof(int32_t), hipMemcpyHostToDevice, st));
  if (cols) {
    const ot::ColP C = col_params(c);
    HIPCHK(ot::launch_eval_cols(fp64, T, E, C, P<int64_t>(c->loff), P<double4>(c->lrec), P<int32_t>(c->lid),
                                P<double>(c->lh), phi, acc, npix, tau, c->p.G,
                                ot::cols_lds_cpw(C.npix, fp64, C.nthr), false, nullptr, st,
                                P<int32_t>(c->abu_blist), nup));
  } else if (fp64)
    HIPCHK(ot::launch_eval64(T, E, P<int64_t>(c->loff), P<double4>(c->lrec), (double *)phi, (double *)acc, c->p.G,
                             st, P<int32_t>(c->abu_blist), nup));
  else
    HIPCHK(ot::launch_eval32(T, E, P<int64_t>(c->loff), P<double4>(c->lrec), P<int32_t>(c->lid), (float *)phi,
                             (float *)acc, c->p.G, st, P<int32_t>(c->abu_blist), nup));
  HIPCHK(hipEventRecord(c->ev[2], st));
  c->off_host.resize(nb + 1);
  HIPCHK(hipMemcpyAsync(c->off_host.data(), c->loff.ptr, (nb + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));  // also keeps blist alive until its copy is done
  c->lists_valid = true;
  if (stats) {
    list_stats(c, std::vector<int32_t>(), stats);
    int64_t tot_up = 0;
    for (int64_t b = 0; b < nb; ++b)
      if (flag[b]) tot_up += c->off_host[b + 1] - c->off_host[b] - 1;
    stats->n_interactions = 512 * tot_up;  // pairs of the blocks evaluated in full
    stats->a_lim_used = alim;
    stats->ms_list = elapsed(c->ev[0], c->ev[1]);
    stats->ms_eval = elapsed(c->ev[1], c->ev[2]);
    stats->ms_build = c->ms_build;
    stats->ewald_used = OT_EWALD_TABLE;
  }
  return OT_OK;
}

// The walk at arbitrary target points (Sec. 2.1): a list per point with the
// MAC suite at the point, then the FP64 pair kernels of the cell walks.
ot_status points_impl(ot_ctx *c, int64_t n, const double *xyz, double *phi, double *acc, ot_stats *stats,
                      void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  c->npts = 0;  // the previous call's lists are gone whatever happens below
  if (n < 0) return fail(c, OT_ERR_INVALID_ARG, "n must be >= 0");
  if (n > ((int64_t)1 << 31)) return fail(c, OT_ERR_INVALID_ARG, "at most 2^31 target points per call");
  if (n > 0 && (!xyz || !phi || !acc)) return fail(c, OT_ERR_INVALID_ARG, "xyz, phi and acc must be device pointers");
  if (!c->built) return fail(c, OT_ERR_STATE, "ot_solve_points before a successful ot_build");
  if (stats) memset(stats, 0, sizeof(*stats));
  if (n == 0) return OT_OK;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->p.device));
  // every point inside the domain: its offsets to the nodes then stay within
  // the box on every isolated axis (the Ewald table's range).  Checked on the
  // device; the host reads one index per checking workgroup.
  {
    ot::Box3 box;
    for (int k = 0; k < 3; ++k) {
      box.lo[k] = c->p.origin[k];
      box.hi[k] = c->p.origin[k] + c->p.nroot[k] * c->p.root_size;
    }
    const int cgrid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    OTCHK(dalloc(c, c->pcheck, (size_t)cgrid * sizeof(int64_t)));
    HIPCHK(ot::launch_points_check(xyz, n, box, cgrid, P<int64_t>(c->pcheck), st));
    std::vector<int64_t> first(cgrid);
    HIPCHK(hipMemcpyAsync(first.data(), c->pcheck.ptr, first.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int64_t bad = *std::min_element(first.begin(), first.end());
    if (bad < n) return fail(c, OT_ERR_INVALID_ARG, "target point " + std::to_string(bad) + " is not inside the domain");
  }
  if (c->bctype != ot::BC_ISO) {
    if (c->p.ewald == OT_EWALD_EXACT)
      return fail(c, OT_ERR_UNSUPPORTED, "per-pair exact Ewald series is not built into the walk");
    OTCHK(ewald_prepare(c, nullptr, st));
  }
  double alim = 0.0;
  if (c->p.mac == OT_MAC_APE || c->p.mac == OT_MAC_MPE) OTCHK(ape_limit(c, st, &alim));
  for (int i = 0; i < 3; ++i)
    if (!c->ev[i]) HIPCHK(hipEventCreate(&c->ev[i]));
  const ot::Topology &t = c->topo;
  ot::DevTree T = dev_tree(c);
  const ot::MacP mp = mac_params(c, c->p.mac, alim, false);
  int64_t capA = 0;
  for (int l = 1; l <= t.lmax; ++l) capA = std::max(capA, t.level_begin[l + 1] - t.level_begin[l]);
  const int64_t stride = 2 * capA + 9 * t.nb;
  // one single-wave workgroup per point in flight, each with its own
  // traversal scratch (sized for the worst case, every node opened)
  int64_t grid = std::min<int64_t>(n, 8192);
  const int64_t budget = (int64_t)4 << 30;  // scratch bytes
  while (grid > 64 && grid * stride * 4 > budget) grid /= 2;
  OTCHK(dalloc(c, c->lscratch, (size_t)(grid * stride * 4)));
  OTCHK(dalloc(c, c->pcount, n * sizeof(int32_t)));
  OTCHK(dalloc(c, c->pnodes, 2 * n * sizeof(int32_t)));
  OTCHK(dalloc(c, c->poff, (n + 1) * sizeof(int64_t)));
  HIPCHK(hipEventRecord(c->ev[0], st));
  HIPCHK(ot::launch_lists(false, T, mp, (int)grid, P<int32_t>(c->pcount), P<int32_t>(c->pnodes), nullptr, nullptr,
                          nullptr, nullptr, P<int32_t>(c->lscratch), stride, capA, st, xyz, n));
  HIPCHK(ot::launch_scan(P<int32_t>(c->pcount), n, P<int64_t>(c->poff), st));
  int64_t total = 0;
  HIPCHK(hipMemcpyAsync(&total, P<int64_t>(c->poff) + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  OTCHK(dalloc(c, c->prec, (size_t)total * sizeof(double4)));
  OTCHK(dalloc(c, c->pid, (size_t)total * sizeof(int32_t)));
  HIPCHK(ot::launch_lists(true, T, mp, (int)grid, P<int32_t>(c->pcount), nullptr, P<int64_t>(c->poff),
                          P<double4>(c->prec), P<int32_t>(c->pid), nullptr, P<int32_t>(c->lscratch), stride, capA,
                          st, xyz, n));
  HIPCHK(hipEventRecord(c->ev[1], st));
  HIPCHK(ot::launch_eval_points64(ewald_desc(c), n, xyz, P<int64_t>(c->poff), P<double4>(c->prec), phi, acc,
                                  c->p.G, st));
  HIPCHK(hipEventRecord(c->ev[2], st));
  c->poff_host.resize(n + 1);
  HIPCHK(hipMemcpyAsync(c->poff_host.data(), c->poff.ptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  std::vector<int32_t> nodes;
  if (stats) {
    nodes.resize(2 * n);
    HIPCHK(hipMemcpyAsync(nodes.data(), c->pnodes.ptr, nodes.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  c->npts = n;
  if (stats) {
    int64_t mx = 0;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t len = c->poff_host[i + 1] - c->poff_host[i];
      mx = std::max(mx, len);
      int k = 0;
      while (k < 31 && ((int64_t)2 << k) <= len) ++k;
      ++stats->list_hist[k];
      stats->n_opened += nodes[2 * i];
      stats->n_accepted += len - nodes[2 * i + 1];
    }
    stats->total_list = total;
    stats->max_list = mx;
    stats->n_interactions = total;
    stats->a_lim_used = alim;
    stats->ms_build = c->ms_build;
    stats->ms_list = elapsed(c->ev[0], c->ev[1]);
    stats->ms_eval = elapsed(c->ev[1], c->ev[2]);
    stats->ewald_used = OT_EWALD_TABLE;
  }
  return OT_OK;
}

}  // namespace

extern "C" {

ot_status ot_solve_points(ot_ctx *c, int64_t n, const double *xyz, double *phi, double *acc, ot_stats *stats,
                          void *stream) {
  return points_impl(c, n, xyz, phi, acc, stats, stream);
}

ot_status ot_export_point_list(ot_ctx *c, int64_t i, int32_t *ids, int64_t cap, int64_t *len) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (!len) return fail(c, OT_ERR_INVALID_ARG, "len must not be null");
  if (i < 0 || i >= c->npts) return fail(c, OT_ERR_INVALID_ARG, "no such target point in the last ot_solve_points");
  const int64_t o0 = c->poff_host[i], o1 = c->poff_host[i + 1];
  *len = o1 - o0;
  if (ids && cap > 0) {
    const int64_t m = std::min(cap, o1 - o0);
    HIPCHK(hipSetDevice(c->p.device));
    HIPCHK(hipMemcpy(ids, P<int32_t>(c->pid) + o0, m * sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  return OT_OK;
}

ot_status ot_solve_abu(ot_ctx *c, float *phi, float *acc, float *npix, float *tau, double tol, double tol_tau,
                       int32_t *updated_host, ot_stats *stats, void *stream) {
  return abu_impl(c, false, phi, acc, npix, tau, tol, tol_tau, updated_host, stats, stream);
}

ot_status ot_solve_abu64(ot_ctx *c, double *phi, double *acc, double *npix, double *tau, double tol,
                         double tol_tau, int32_t *updated_host, ot_stats *stats, void *stream) {
  return abu_impl(c, true, phi, acc, npix, tau, tol, tol_tau, updated_host, stats, stream);
}

void ot_params_default(ot_params *p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->nroot[0] = p->nroot[1] = p->nroot[2] = 1;
  p->root_size = 1.0;
  p->G = 1.0;
  p->theta_lim = 0.5;
  p->eta_sb = 1.2;
  p->mac = OT_MAC_BH;
  p->ewald = OT_EWALD_TABLE;
  p->a_lim = 0.0;
  p->eps_lim = 1e-3;
  p->ewald_n = 64;
  p->device = 0;
  p->nside = 0;
  p->il_ntheta = 25;
  p->il_nphi = 50;
  p->il_npsi = 25;
  p->il_nr = 50;
  p->il_nazi = 100;
  p->theta_pix = 0.0;
  p->kappa = 1.0;
  p->max_dist = 1e99;
  p->psi_max = 0.98;
  p->mlp_reach = 1.0;
  p->list_group = 8;
}

ot_status ot_create(const ot_params *p, ot_ctx **out) {
  if (!p || !out) return OT_ERR_INVALID_ARG;
  *out = nullptr;
  ot_ctx *c = new (std::nothrow) ot_ctx();
  if (!c) return OT_ERR_OOM;
  c->p = *p;
  auto bad = [&](const char *m) {
    // keep the context so the caller can read the message, then let them destroy it
    c->err = m;
    *out = c;
    return OT_ERR_INVALID_ARG;
  };
  for (int k = 0; k < 3; ++k) {
    if (p->nroot[k] < 1) return bad("nroot must be >= 1");
    if (p->bc[k] != 0 && p->bc[k] != 1) return bad("bc must be 0 (isolated) or 1 (periodic)");
    c->box[k] = p->nroot[k] * p->root_size;
  }
  if (!std::isfinite(p->mlp_reach)) return bad("mlp_reach must be finite");
  if (p->list_group != 0 && p->list_group != 4 && p->list_group != 8) return bad("list_group must be 0, 4 or 8");
  if (!(p->root_size > 0) || !std::isfinite(p->root_size)) return bad("root_size must be > 0");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(p->origin[k])) return bad("origin must be finite");
  if (!(p->G > 0) || !std::isfinite(p->G)) return bad("G must be > 0");
  if (!(p->theta_lim > 0) || !std::isfinite(p->theta_lim)) return bad("theta_lim must be > 0");
  if (!(p->eta_sb >= 0) || !std::isfinite(p->eta_sb)) return bad("eta_sb must be >= 0");
  if (p->mac != OT_MAC_BH && p->mac != OT_MAC_APE && p->mac != OT_MAC_MPE) return bad("unknown MAC");
  if (p->ewald != OT_EWALD_TABLE && p->ewald != OT_EWALD_EXACT && p->ewald != OT_EWALD_MLP)
    return bad("unknown Ewald mode");
  if (p->mac != OT_MAC_BH && !(p->a_lim > 0) && !(p->eps_lim > 0)) return bad("APE/MPE need a_lim > 0 or eps_lim > 0");
  if (p->ewald_n < 2 || p->ewald_n > 512) return bad("ewald_n must be in [2, 512]");
  if (p->nside != 0 && p->nside != 1 && p->nside != 2 && p->nside != 4) return bad("nside must be 0, 1, 2 or 4");
  if (p->nside) {
    if (p->il_ntheta < 1 || p->il_nphi < 1 || p->il_npsi < 1 || p->il_nr < 1 || p->il_nazi < 1)
      return bad("intersection-table sizes must be >= 1");
    if (p->il_nr > 256 || (int64_t)p->il_nr * p->il_nazi > 8192)
      return bad("intersection table: il_nr <= 256 and il_nr * il_nazi <= 8192");
    if (p->il_ntheta > 64 || p->il_npsi > 64 || p->il_nphi > 128 || (p->il_nphi & 1))
      return bad("intersection table: ntheta, npsi <= 64 and an even nphi <= 128");
    if (!(p->psi_max > 0) || !(p->kappa >= 0) || !(p->max_dist > 0)) return bad("bad column parameters");
  }
  const int nper = p->bc[0] + p->bc[1] + p->bc[2];
  if (nper == 0) c->bctype = ot::BC_ISO;
  else if (nper == 3) c->bctype = ot::BC_3P;
  else if (p->bc[0] && p->bc[1] && !p->bc[2]) {
    // the far-field limit replaces the series beyond |dz| = 2 Lx, where the
    // dropped Fourier modes decay as exp(-2 pi |dz| / Ly): below 1e-5 of the
    // kernel only while Ly <= Lx
    if (c->box[1] > c->box[0]) {
      c->err = "2P1I needs Ly <= Lx (the far-field switch at |dz| = 2 Lx)";
      *out = c;
      return OT_ERR_UNSUPPORTED;
    }
    c->bctype = ot::BC_2P1I;
  }
  else if (p->bc[0] && !p->bc[1] && !p->bc[2]) c->bctype = ot::BC_1P2I;
  else {
    c->err = "boundary combination not supported (isolated, 3P, x,y-periodic 2P1I and x-periodic 1P2I are)";
    *out = c;
    return OT_ERR_UNSUPPORTED;
  }
  *out = c;
  return OT_OK;
}

ot_status ot_set_blocks(ot_ctx *c, int64_t nb, const int32_t *level, const int32_t *coord) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (nb <= 0 || !level || !coord) return fail(c, OT_ERR_INVALID_ARG, "need nb > 0 and host level/coord arrays");
  ot::Topology t;
  std::string why = ot::build_topology(c->p.nroot, nb, level, coord, t);
  if (!why.empty()) return fail(c, OT_ERR_BAD_GRID, why);
  if (t.na + 584 * t.nb >= ((int64_t)1 << 31))
    return fail(c, OT_ERR_UNSUPPORTED, "more than 2^31 tree nodes");
  c->topo = std::move(t);
  c->have_blocks = true;
  c->dev_topo = false;
  c->built = false;
  c->lists_valid = false;
  c->npts = 0;
  c->alim_valid = false;
  return OT_OK;
}

ot_status ot_build(ot_ctx *c, const double *rho, void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (!c->have_blocks) return fail(c, OT_ERR_STATE, "ot_build before ot_set_blocks");
  if (!rho) return fail(c, OT_ERR_INVALID_ARG, "rho must be a device pointer");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->p.device));
  c->built = false;
  c->lists_valid = false;
  c->npts = 0;
  c->alim_valid = false;
  if (!c->dev_topo) OTCHK(upload_topology(c, st));
  for (int i = 0; i < 4; ++i)
    if (!c->ev[i]) HIPCHK(hipEventCreate(&c->ev[i]));
  int bad = 0;
  HIPCHK(hipMemsetAsync(c->flag.ptr, 0, sizeof(int), st));
  HIPCHK(hipEventRecord(c->ev[0], st));
  ot::DevTree T = dev_tree(c);
  HIPCHK(ot::launch_build(T, rho, P<int>(c->flag), c->topo.level_begin, c->topo.lmax, st));
  if (c->p.mac == OT_MAC_MPE)
    HIPCHK(ot::launch_mpe(T, c->mpe_npairs, P<int32_t>(c->mpe_pnode), P<int32_t>(c->mpe_pblock),
                          P<int64_t>(c->mpe_poff), P<double2>(c->mpe_part), st));
  HIPCHK(hipEventRecord(c->ev[3], st));
  HIPCHK(hipMemcpyAsync(&bad, c->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  c->ms_build = elapsed(c->ev[0], c->ev[3]);
  if (bad) return fail(c, OT_ERR_NUMERIC, "density must be finite and >= 0");
  c->built = true;
  return OT_OK;
}

ot_status ot_solve(ot_ctx *c, float *phi, float *acc, float *npix, float *tau, ot_stats *stats,
                   void *stream) {
  return solve_impl(c, false, phi, acc, npix, tau, stats, stream);
}

ot_status ot_solve64(ot_ctx *c, double *phi, double *acc, double *npix, double *tau, ot_stats *stats,
                     void *stream) {
  return solve_impl(c, true, phi, acc, npix, tau, stats, stream);
}

ot_status ot_export_raytable(ot_ctx *c, int64_t *nentries, int64_t *npairs, int64_t *off, int32_t *pix,
                             double *w, void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  OTCHK(raytable_prepare(c, (hipStream_t)stream));
  const ot::RayTableP RP = raytable_desc(c);
  if (nentries) *nentries = RP.nentries;
  if (npairs) *npairs = c->rt_pairs;
  if (off) HIPCHK(hipMemcpy(off, c->rt_off.ptr, (RP.nentries + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (w) HIPCHK(hipMemcpy(w, c->rt_w64.ptr, c->rt_pairs * sizeof(double), hipMemcpyDeviceToHost));
  if (pix) {
    std::vector<uint16_t> p16(c->rt_pairs);
    HIPCHK(hipMemcpy(p16.data(), c->rt_pix.ptr, c->rt_pairs * sizeof(uint16_t), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < c->rt_pairs; ++i) pix[i] = p16[i];
  }
  return OT_OK;
}

ot_status ot_ewald_prepare(ot_ctx *c, const char *cache_path, void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  return ewald_prepare(c, cache_path, (hipStream_t)stream);
}

int64_t ot_num_amr_nodes(const ot_ctx *c) { return c && c->have_blocks ? c->topo.na : -1; }

ot_status ot_export_topology(const ot_ctx *cc, int32_t *level, int32_t *coord, int64_t *leaf,
                             int64_t *child, uint64_t *key) {
  ot_ctx *c = const_cast<ot_ctx *>(cc);
  if (!c) return OT_ERR_INVALID_ARG;
  if (!c->have_blocks) return fail(c, OT_ERR_STATE, "no blocks set");
  const ot::Topology &t = c->topo;
  if (level) memcpy(level, t.alev.data(), t.na * sizeof(int32_t));
  if (coord) memcpy(coord, t.acoord.data(), 3 * t.na * sizeof(int32_t));
  if (leaf) memcpy(leaf, t.aleaf.data(), t.na * sizeof(int64_t));
  if (child) memcpy(child, t.achild.data(), 8 * t.na * sizeof(int64_t));
  if (key) memcpy(key, t.akey.data(), t.na * sizeof(uint64_t));
  return OT_OK;
}

ot_status ot_export_moments(ot_ctx *c, double *M, double *com) {
  if (!c) return OT_ERR_INVALID_ARG;
  if (!c->built) return fail(c, OT_ERR_STATE, "no tree built");
  if (!M || !com) return fail(c, OT_ERR_INVALID_ARG, "null output");
  HIPCHK(hipSetDevice(c->p.device));
  const ot::Topology &t = c->topo;
  std::vector<double4> a(t.na), bt(72 * t.nb);
  std::vector<double> cm(512 * t.nb);
  HIPCHK(hipMemcpy(a.data(), c->amc.ptr, t.na * sizeof(double4), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(bt.data(), c->btmc.ptr, 72 * t.nb * sizeof(double4), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(cm.data(), c->cm.ptr, 512 * t.nb * sizeof(double), hipMemcpyDeviceToHost));
  auto put = [&](int64_t id, const double4 &v) {
    M[id] = v.w;
    com[3 * id] = v.x;
    com[3 * id + 1] = v.y;
    com[3 * id + 2] = v.z;
  };
  for (int64_t i = 0; i < t.na; ++i) put(i, a[i]);
  for (int64_t lb = 0; lb < t.nb; ++lb) {
    for (int o = 0; o < 8; ++o) put(t.na + 8 * lb + o, bt[72 * lb + o]);
    for (int q = 0; q < 64; ++q) put(t.na + 8 * t.nb + 64 * lb + q, bt[72 * lb + 8 + q]);
    const double h = ot::size_at(c->p.root_size, t.blev[lb]) / 8.0;
    for (int ci = 0; ci < 512; ++ci) {
      const int ijk[3] = {ci & 7, (ci >> 3) & 7, ci >> 6};
      double4 v;
      double x[3];
      for (int k = 0; k < 3; ++k)
        x[k] = ot::centre_coord(c->p.origin[k], 8 * (int64_t)t.bcoord[3 * lb + k] + ijk[k], h);
      v.x = x[0];
      v.y = x[1];
      v.z = x[2];
      v.w = cm[512 * lb + ci];
      put(t.na + 72 * t.nb + 512 * lb + ci, v);
    }
  }
  return OT_OK;
}

ot_status ot_export_list(ot_ctx *c, int64_t b, int32_t *ids, int64_t cap, int64_t *len) {
  if (!c) return OT_ERR_INVALID_ARG;
  if (!c->lists_valid) return fail(c, OT_ERR_STATE, "no lists: call ot_solve first");
  const int64_t ntg = c->list_sub ? 8 * c->topo.nb : c->topo.nb;
  if (b < 0 || b >= ntg || !len) return fail(c, OT_ERR_INVALID_ARG, "bad list index");
  const int64_t n = c->off_host[b + 1] - c->off_host[b];
  *len = n;
  if (ids && cap > 0) {
    HIPCHK(hipSetDevice(c->p.device));
    HIPCHK(hipMemcpy(ids, P<int32_t>(c->lid) + c->off_host[b], std::min(n, cap) * sizeof(int32_t),
                     hipMemcpyDeviceToHost));
  }
  return OT_OK;
}

ot_status ot_export_ewald_table(ot_ctx *c, double *tab) {
  if (!c) return OT_ERR_INVALID_ARG;
  if (!c->ewald_ready) return fail(c, OT_ERR_STATE, "no Ewald table");
  if (!tab) return fail(c, OT_ERR_INVALID_ARG, "null output");
  HIPCHK(hipSetDevice(c->p.device));
  const size_t np = (size_t)c->ew_n * c->ew_n * c->ew_n;
  HIPCHK(hipMemcpy(tab, c->tab64.ptr, np * 10 * sizeof(double), hipMemcpyDeviceToHost));
  return OT_OK;
}

void ot_mlp_config_default(ot_mlp_config *cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->nsamples = 1 << 21;
  cfg->nval = 100000;
  cfg->epochs = 300;
  cfg->batch = 2048;
  cfg->lr_max = 3e-3;
  cfg->lr_min = 1e-5;
  cfg->seed = 4;
  cfg->tol = 5e-3;
}

namespace {

// every input the trained surrogate depends on (the training recipe's
// version in i[12]: bump it when the training changes)
ot::CacheKey mlp_key(const ot_ctx *c, const ot_mlp_config *cfg) {
  ot::CacheKey k;
  memset(&k, 0, sizeof(k));
  k.kind = 2;
  k.i[0] = c->bctype;
  k.i[1] = ot::mlpdef::NP;
  k.i[2] = ot::mlpdef::NO;
  k.i[3] = OT_MLP_NNORM;
  k.i[4] = cfg->nsamples;
  k.i[5] = cfg->nval;
  k.i[6] = cfg->epochs;
  k.i[7] = cfg->batch;
  memcpy(&k.i[8], &cfg->seed, sizeof(cfg->seed));
  k.i[9] = c->ew_n;
  k.i[10] = c->ew_rcut2;
  k.i[11] = c->ew_fcut2;
  k.i[12] = 1;
  k.d[0] = cfg->lr_max;
  k.d[1] = cfg->lr_min;
  k.d[2] = cfg->tol;
  k.d[3] = c->ew_alpha;
  for (int q = 0; q < 3; ++q) {
    k.d[4 + q] = c->box[q];
    k.d[7 + q] = c->ew_ext[q];
  }
  return k;
}

struct MlpFile {
  float params[ot::mlpdef::NP];
  double norm[OT_MLP_NNORM];
  ot_mlp_report report;
};

ot_status mlp_train_impl(ot_ctx *c, const ot_mlp_config *cfg, ot_mlp_report *rep, hipStream_t st);

}  // namespace

ot_status ot_mlp_train(ot_ctx *c, const ot_mlp_config *cfg, const char *cache_path, ot_mlp_report *rep,
                       void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (!cfg) return fail(c, OT_ERR_INVALID_ARG, "null config");
  if (c->bctype == ot::BC_1P2I)
    return fail(c, OT_ERR_UNSUPPORTED, "the learned surrogate covers 3P and 2P1I (1P2I uses the table)");
  if (c->bctype == ot::BC_ISO) return fail(c, OT_ERR_STATE, "the surrogate needs periodic or mixed boundaries");
  if (cfg->nsamples < 32 || cfg->nsamples % 32 || cfg->batch < 32 || cfg->batch % 32 ||
      cfg->batch > cfg->nsamples || cfg->epochs < 1 || cfg->nval < 1 || !(cfg->lr_max > 0) ||
      !(cfg->lr_min >= 0) || !(cfg->tol > 0))
    return fail(c, OT_ERR_INVALID_ARG,
                "surrogate training needs nsamples, batch multiples of 32 with batch <= nsamples, "
                "epochs >= 1, nval >= 1, lr_max > 0, lr_min >= 0, tol > 0");
  if (cfg->nsamples > ((int64_t)1 << 28) || cfg->nval > ((int64_t)1 << 26))
    return fail(c, OT_ERR_INVALID_ARG, "nsamples <= 2^28 and nval <= 2^26");
  std::string why;
  if (cache_path && !ot::cache_path_usable(cache_path, why)) return fail(c, OT_ERR_IO, why);
  if (!c->ewald_ready) ewald_params(c);
  const ot::CacheKey key = mlp_key(c, cfg);
  hipStream_t st = (hipStream_t)stream;
  if (cache_path) {
    std::vector<char> payload;
    const ot::CacheRead cr = ot::cache_read(cache_path, key, payload, why);
    if (cr == ot::CacheRead::IoError) return fail(c, OT_ERR_IO, why);
    if (cr == ot::CacheRead::Loaded && payload.size() == sizeof(MlpFile)) {
      const MlpFile *f = reinterpret_cast<const MlpFile *>(payload.data());
      HIPCHK(hipSetDevice(c->p.device));
      OTCHK(ewald_prepare(c, nullptr, st));
      OTCHK(dalloc(c, c->mlp_P, ot::mlpdef::NP * sizeof(float)));
      HIPCHK(hipMemcpyAsync(c->mlp_P.ptr, f->params, sizeof(f->params), hipMemcpyHostToDevice, st));
      memcpy(c->mlp_norm, f->norm, sizeof(c->mlp_norm));
      c->mlp_have = true;
      OTCHK(mlp_pack(c, st));
      HIPCHK(hipStreamSynchronize(st));
      c->mlp_ok = f->report.ok != 0;
      if (rep) {
        *rep = f->report;
        rep->ms_samples = rep->ms_train = rep->ms_validate = 0.0;
        rep->from_cache = 1;
      }
      return OT_OK;
    }
  }
  ot_mlp_report local;
  OTCHK(mlp_train_impl(c, cfg, &local, st));
  if (rep) *rep = local;
  if (cache_path) {
    MlpFile f;
    memset(&f, 0, sizeof(f));
    HIPCHK(hipMemcpy(f.params, c->mlp_P.ptr, sizeof(f.params), hipMemcpyDeviceToHost));
    memcpy(f.norm, c->mlp_norm, sizeof(f.norm));
    f.report = local;
    if (!ot::cache_write(cache_path, key, &f, sizeof(f), why)) return fail(c, OT_ERR_IO, why);
  }
  return OT_OK;
}

namespace {

ot_status mlp_train_impl(ot_ctx *c, const ot_mlp_config *cfg, ot_mlp_report *rep, hipStream_t st) {
  using namespace ot::mlpdef;
  HIPCHK(hipSetDevice(c->p.device));
  OTCHK(ewald_prepare(c, nullptr, st));
  c->mlp_ok = false;
  const int64_t n = cfg->nsamples, nv = cfg->nval;
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto ms = [](auto a, auto b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
  // training offsets and their series values
  auto t0 = now();
  Scoped u(c), ser(c), x(c), t(c), m(c), v(c), losses(c);
  OTCHK(dalloc(c, u.b, (size_t)n * 3 * sizeof(double)));
  OTCHK(dalloc(c, ser.b, (size_t)n * 10 * sizeof(double)));
  HIPCHK(ot::launch_mlp_points(cfg->seed * 3 + 1, n, c->ew_ext, u.p<double>(), st));
  const ot::EwaldP E = ewald_desc(c);
  HIPCHK(ot::launch_ewald_points(E, c->ew_alpha, c->ew_rcut2, c->ew_fcut2, n, u.p<double>(), ser.p<double>(), st));
  // scaling: inputs to [-1, 1]; outputs standardised on the first offsets
  const int64_t ns = std::min<int64_t>(n, 65536);
  std::vector<double> hs((size_t)ns * 10);
  HIPCHK(hipMemcpyAsync(hs.data(), ser.b.ptr, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // outputs standardised by mean and standard deviation; the second
  // derivatives by 3 standard deviations, which weighs them 1/9 in the loss:
  // the walk multiplies them by offsets within half a table spacing
  for (int k = 0; k < 3; ++k) c->mlp_norm[k] = c->ew_ext[k];
  for (int o = 0; o < NO; ++o) {
    double s1 = 0.0, s2 = 0.0;
    for (int64_t q = 0; q < ns; ++q) s1 += hs[10 * q + o];
    const double mu = s1 / (double)ns;
    for (int64_t q = 0; q < ns; ++q) s2 += (hs[10 * q + o] - mu) * (hs[10 * q + o] - mu);
    const double sig = std::sqrt(s2 / (double)ns);
    c->mlp_norm[3 + o] = mu;
    c->mlp_norm[3 + NO + o] = (sig > 0 ? sig : 1.0) * (o < 4 ? 1.0 : 3.0);
  }
  OTCHK(dalloc(c, x.b, (size_t)n * 3 * sizeof(float)));
  OTCHK(dalloc(c, t.b, (size_t)n * NO * sizeof(float)));
  HIPCHK(ot::launch_mlp_prepare(n, u.p<double>(), ser.p<double>(), mlp_norm_of(c), x.p<float>(), t.p<float>(), st));
  HIPCHK(hipStreamSynchronize(st));
  release(c, ser.b);
  release(c, u.b);
  auto t1 = now();
  // Adam with a cosine step size; each epoch starts at a different offset
  const int64_t spe = n / cfg->batch, total = spe * cfg->epochs;
  OTCHK(dalloc(c, c->mlp_P, NP * sizeof(float)));
  OTCHK(dalloc(c, m.b, NP * sizeof(float)));
  OTCHK(dalloc(c, v.b, NP * sizeof(float)));
  OTCHK(dalloc(c, losses.b, (size_t)total * sizeof(float)));
  OTCHK(mlp_grad_scratch(c, cfg->batch));
  HIPCHK(hipMemsetAsync(m.b.ptr, 0, NP * sizeof(float), st));
  HIPCHK(hipMemsetAsync(v.b.ptr, 0, NP * sizeof(float), st));
  HIPCHK(ot::launch_mlp_init(cfg->seed * 3, P<float>(c->mlp_P), st));
  c->mlp_have = false;
  uint64_t rot = cfg->seed * 0x9E3779B97F4A7C15ull + 12345;
  int64_t step = 0;
  for (int e = 0; e < cfg->epochs; ++e) {
    rot ^= rot << 13;
    rot ^= rot >> 7;
    rot ^= rot << 17;
    const int64_t s0 = (int64_t)(rot % (uint64_t)(n / 32)) * 32;
    for (int64_t k = 0; k < spe; ++k, ++step) {
      const double lr = cfg->lr_min + 0.5 * (cfg->lr_max - cfg->lr_min) *
                                          (1.0 + std::cos(M_PI * (double)step / (double)total));
      HIPCHK(ot::launch_mlp_step(P<float>(c->mlp_P), n, (s0 + k * cfg->batch) % n, cfg->batch, x.p<float>(),
                                 t.p<float>(), P<float>(c->mlp_part), P<float>(c->mlp_lossp),
                                 losses.p<float>() + step, m.p<float>(), v.p<float>(), (float)lr,
                                 (int)std::min<int64_t>(step + 1, 1 << 30), st));
    }
  }
  std::vector<float> hl((size_t)total);
  HIPCHK(hipMemcpyAsync(hl.data(), losses.b.ptr, hl.size() * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  release(c, x.b);
  release(c, t.b);
  c->mlp_have = true;
  OTCHK(mlp_pack(c, st));
  auto t2 = now();
  // held-out validation against the series, with the table alongside
  Scoped d(c), ex(c), ml(c), tb(c);
  OTCHK(dalloc(c, d.b, (size_t)nv * 3 * sizeof(double)));
  OTCHK(dalloc(c, ex.b, (size_t)nv * NO * sizeof(double)));
  OTCHK(dalloc(c, ml.b, (size_t)nv * NO * sizeof(double)));
  OTCHK(dalloc(c, tb.b, (size_t)nv * NO * sizeof(double)));
  HIPCHK(ot::launch_mlp_points(cfg->seed * 3 + 2, nv, c->ew_ext, d.p<double>(), st));
  OTCHK(ewald_points(c, OT_EWALD_EXACT, nv, d.p<double>(), ex.p<double>(), st));
  OTCHK(ewald_points(c, OT_EWALD_MLP, nv, d.p<double>(), ml.p<double>(), st));
  OTCHK(ewald_points(c, OT_EWALD_TABLE, nv, d.p<double>(), tb.p<double>(), st));
  std::vector<double> hx((size_t)nv * NO), hm((size_t)nv * NO), ht((size_t)nv * NO);
  HIPCHK(hipMemcpyAsync(hx.data(), ex.b.ptr, hx.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hm.data(), ml.b.ptr, hm.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(ht.data(), tb.b.ptr, ht.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // accepted when phi_c and A_c are within tol of their largest value and the
  // second derivatives, which the walk multiplies by offsets within half a
  // table spacing, within 10 tol
  double em[NO], et[NO];
  bool ok = true;
  for (int o = 0; o < NO; ++o) {
    double mx = 0.0, dm = 0.0, dt = 0.0;
    for (int64_t q = 0; q < nv; ++q) {
      mx = std::max(mx, std::fabs(hx[NO * q + o]));
      dm = std::max(dm, std::fabs(hm[NO * q + o] - hx[NO * q + o]));
      dt = std::max(dt, std::fabs(ht[NO * q + o] - hx[NO * q + o]));
    }
    em[o] = mx > 0 ? dm / mx : dm;
    et[o] = mx > 0 ? dt / mx : dt;
    if (!(em[o] <= (o < 4 ? 1.0 : 10.0) * cfg->tol)) ok = false;
  }
  c->mlp_ok = ok;
  auto t3 = now();
  if (rep) {
    memset(rep, 0, sizeof(*rep));
    double a = 0.0, b = 0.0;
    for (int64_t k = 0; k < spe; ++k) {
      a += hl[k];
      b += hl[total - spe + k];
    }
    rep->loss_first = a / (double)spe;
    rep->loss_last = b / (double)spe;
    for (int o = 0; o < NO; ++o) {
      rep->err_mlp[o] = em[o];
      rep->err_table[o] = et[o];
    }
    rep->ms_samples = ms(t0, t1);
    rep->ms_train = ms(t1, t2);
    rep->ms_validate = ms(t2, t3);
    rep->ok = ok ? 1 : 0;
  }
  return OT_OK;
}

}  // namespace

ot_status ot_mlp_get(ot_ctx *c, float *params, double *norm) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (!c->mlp_have) return fail(c, OT_ERR_STATE, "no surrogate: train or set one first");
  HIPCHK(hipSetDevice(c->p.device));
  if (params) HIPCHK(hipMemcpy(params, c->mlp_P.ptr, ot::mlpdef::NP * sizeof(float), hipMemcpyDeviceToHost));
  if (norm) memcpy(norm, c->mlp_norm, sizeof(c->mlp_norm));
  return OT_OK;
}

ot_status ot_mlp_set(ot_ctx *c, const float *params, const double *norm, int32_t accept, void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (!params || !norm) return fail(c, OT_ERR_INVALID_ARG, "null parameters or scaling");
  if (c->bctype == ot::BC_1P2I)
    return fail(c, OT_ERR_UNSUPPORTED, "the learned surrogate covers 3P and 2P1I (1P2I uses the table)");
  for (int k = 0; k < OT_MLP_NNORM; ++k)
    if (!std::isfinite(norm[k]) || ((k < 3 || k >= 3 + ot::mlpdef::NO) && !(norm[k] > 0)))
      return fail(c, OT_ERR_INVALID_ARG, "scaling must be finite with ext > 0 and sig > 0");
  for (int i = 0; i < ot::mlpdef::NP; ++i)
    if (!std::isfinite(params[i])) return fail(c, OT_ERR_INVALID_ARG, "non-finite parameter");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->p.device));
  OTCHK(dalloc(c, c->mlp_P, ot::mlpdef::NP * sizeof(float)));
  HIPCHK(hipMemcpyAsync(c->mlp_P.ptr, params, ot::mlpdef::NP * sizeof(float), hipMemcpyHostToDevice, st));
  memcpy(c->mlp_norm, norm, sizeof(c->mlp_norm));
  c->mlp_have = true;
  OTCHK(mlp_pack(c, st));
  HIPCHK(hipStreamSynchronize(st));
  c->mlp_ok = accept != 0;
  return OT_OK;
}

ot_status ot_mlp_grad(ot_ctx *c, const float *params, int64_t batch, const float *x, const float *t, float *grad,
                      float *loss, void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (!params || !x || !t || !grad || !loss) return fail(c, OT_ERR_INVALID_ARG, "null pointer");
  if (batch < 32 || batch % 32 || batch > ((int64_t)1 << 24))
    return fail(c, OT_ERR_INVALID_ARG, "batch must be a positive multiple of 32, <= 2^24");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->p.device));
  OTCHK(mlp_grad_scratch(c, batch));
  OTCHK(dalloc(c, c->mlp_loss, sizeof(float)));
  HIPCHK(ot::launch_mlp_grad(params, batch, 0, batch, x, t, P<float>(c->mlp_part), P<float>(c->mlp_lossp), grad,
                             P<float>(c->mlp_loss), st));
  HIPCHK(hipMemcpyAsync(loss, c->mlp_loss.ptr, sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return OT_OK;
}

ot_status ot_mlp_adam_step(ot_ctx *c, float *params, float *m, float *v, int64_t batch, const float *x,
                           const float *t, double lr, int64_t step, float *loss, void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (!params || !m || !v || !x || !t || !loss) return fail(c, OT_ERR_INVALID_ARG, "null pointer");
  if (batch < 32 || batch % 32 || batch > ((int64_t)1 << 24))
    return fail(c, OT_ERR_INVALID_ARG, "batch must be a positive multiple of 32, <= 2^24");
  if (step < 1 || step > ((int64_t)1 << 30)) return fail(c, OT_ERR_INVALID_ARG, "step must be >= 1");
  if (!(lr > 0.0) || !std::isfinite(lr)) return fail(c, OT_ERR_INVALID_ARG, "lr must be finite and > 0");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->p.device));
  OTCHK(mlp_grad_scratch(c, batch));
  OTCHK(dalloc(c, c->mlp_loss, sizeof(float)));
  HIPCHK(ot::launch_mlp_step(params, batch, 0, batch, x, t, P<float>(c->mlp_part), P<float>(c->mlp_lossp),
                             P<float>(c->mlp_loss), m, v, (float)lr, (int)step, st));
  HIPCHK(hipMemcpyAsync(loss, c->mlp_loss.ptr, sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return OT_OK;
}

ot_status ot_mlp_grad_noalloc(ot_ctx *c, const float *params, int64_t batch, const float *x, const float *t,
                              float *grad, float *loss, void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (!params || !x || !t || !grad || !loss) return fail(c, OT_ERR_INVALID_ARG, "null pointer");
  if (batch < 32 || batch % 32)
    return fail(c, OT_ERR_INVALID_ARG, "batch must be a positive multiple of 32");
  if (batch > ot::MLP_NOALLOC_MAX_BATCH)
    return fail(c, OT_ERR_INVALID_ARG,
                "batch " + std::to_string(batch) + " exceeds the fixed workspace of the allocation-free gradient (" +
                    std::to_string(ot::MLP_NOALLOC_MAX_BATCH) + " samples); use ot_mlp_grad");
  float *part = nullptr, *lossp = nullptr;
  hipError_t e = ot::mlp_noalloc_workspace(c->p.device, &part, &lossp);
  if (e != hipSuccess) return dev_fail(c, e, "fixed workspace of the allocation-free gradient");
  HIPCHK(hipSetDevice(c->p.device));
  // every partial and per-workgroup loss is written before it is read:
  // nothing needs clearing between calls
  HIPCHK(ot::launch_mlp_grad(params, batch, 0, batch, x, t, part, lossp, grad, loss, (hipStream_t)stream));
  return OT_OK;
}

ot_status ot_ewald_points(ot_ctx *c, int32_t method, int64_t n, const double *d, double *out, void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (method != OT_EWALD_TABLE && method != OT_EWALD_EXACT && method != OT_EWALD_MLP)
    return fail(c, OT_ERR_INVALID_ARG, "unknown method");
  if (n < 0 || (n > 0 && (!d || !out))) return fail(c, OT_ERR_INVALID_ARG, "bad size or null pointer");
  if (n > ((int64_t)1 << 30)) return fail(c, OT_ERR_INVALID_ARG, "n > 2^30");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->p.device));
  OTCHK(ewald_prepare(c, nullptr, st));
  if (n == 0) return OT_OK;
  OTCHK(ewald_points(c, method, n, d, out, st));
  HIPCHK(hipStreamSynchronize(st));
  return OT_OK;
}

ot_status ot_column_bins(ot_ctx *c, int64_t n, const double *d, const double *h, int32_t *row, void *stream) {
  if (!c) return OT_ERR_INVALID_ARG;
  c->err.clear();
  if (n < 0 || (n > 0 && (!d || !h || !row))) return fail(c, OT_ERR_INVALID_ARG, "bad size or null pointer");
  if (n > ((int64_t)1 << 30)) return fail(c, OT_ERR_INVALID_ARG, "n > 2^30");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->p.device));
  OTCHK(raytable_prepare(c, st));
  HIPCHK(ot::launch_column_bins(col_params(c), n, d, h, row, st));
  HIPCHK(hipStreamSynchronize(st));
  return OT_OK;
}

const char *ot_last_error(const ot_ctx *c) { return c ? c->err.c_str() : "null context"; }

void ot_destroy(ot_ctx *c) {
  if (!c) return;
  if (c->dev_bytes || c->ev[0]) (void)hipSetDevice(c->p.device);
  DevBuf *all[] = {&c->alev, &c->acoord, &c->achild0, &c->aleaf, &c->blev,   &c->bcoord,
                   &c->bamr, &c->amc,    &c->aS,      &c->btmc,  &c->cm,     &c->flag,
                   &c->lcount, &c->lnodes, &c->llat, &c->loff, &c->lrec,    &c->lid,   &c->lscratch, &c->tab64,
                   &c->pcount, &c->pnodes, &c->poff, &c->prec, &c->pid, &c->pcheck,
                   &c->tab32, &c->rt_off, &c->rt_pix, &c->rt_w64, &c->rt_rows, &c->rt_ent, &c->rt_rows8, &c->rt_quad64, &c->mpe_a, &c->mpe_b, &c->mpe_pnode, &c->mpe_pblock, &c->mpe_poff, &c->mpe_part, &c->abu_flag, &c->abu_blist, &c->rt_lut,
                   &c->rt_thr, &c->lh, &c->mlp_P, &c->mlp_pk, &c->mlp_part, &c->mlp_lossp,
                   &c->mlp_loss};
  for (DevBuf *b : all) release(c, *b);
  for (int i = 0; i < 6; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  delete c;
}

}  // extern "C"
