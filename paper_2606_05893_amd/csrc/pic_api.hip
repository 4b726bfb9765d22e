// C ABI of the PIC-MCC library: context set-up on a caller-provided
// workspace, the step driver (deposit -> field -> sources/push/collisions ->
// binning, one stream, one host synchronisation at the end of a step plus
// one per batch of multigrid cycles), and state access.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "pic_ctx.h"

using namespace pic;

namespace {

constexpr size_t kAlign = 256;

struct Carver {
  char* base;
  size_t off;
  template <typename T>
  T* take(long long count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (size_t)(count > 0 ? count : 1) * sizeof(T);
    return p;
  }
};

pic_status set_err(pic_ctx* c, pic_status s, const char* msg) {
  if (c) c->err = msg;
  return s;
}

bool hip_ok(pic_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  if (c) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
  }
  return false;
}

long long pow2_at_least(long long n) {
  long long p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Multigrid hierarchy: halve every axis while all stay even, the coarse
// level keeps at least two z cells, and x, y either stay >= 2 or both reach
// one node (the coarsest 1x1xN level is then solved exactly in z).
int plan_levels(const pic_config* cfg, int dims[16][3]) {
  int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
  int n = 0;
  dims[n][0] = nx; dims[n][1] = ny; dims[n][2] = nz;
  ++n;
  const int limit = cfg->mg_levels > 0 ? std::min(cfg->mg_levels, 16) : 16;
  while (n < limit) {
    if ((nx & 1) || (ny & 1) || (nz & 1)) break;
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    if (cz < 2) break;
    const bool both_one = cx == 1 && cy == 1;
    const bool both_ok = cx >= 2 && cy >= 2;
    if (!both_one && !both_ok) break;
    if (!both_one && ((cx & 1) || (cy & 1))) {
      // Still a valid coarse level for red-black sweeps only if even.
      break;
    }
    nx = cx; ny = cy; nz = cz;
    dims[n][0] = nx; dims[n][1] = ny; dims[n][2] = nz;
    ++n;
    if (both_one) break;
  }
  return n;
}

pic_status validate(const pic_config* c) {
  if (!c) return PIC_ERR_ARG;
  if (c->nx < 2 || c->ny < 2 || c->nz < 2 || (c->nx & 1) || (c->ny & 1) ||
      (c->nz & 1))
    return PIC_ERR_ARG;
  if (!(c->dx > 0.0) || !std::isfinite(c->dx)) return PIC_ERR_ARG;
  if ((c->bc_lo != PIC_BC_DIRICHLET && c->bc_lo != PIC_BC_NEUMANN) ||
      (c->bc_hi != PIC_BC_DIRICHLET && c->bc_hi != PIC_BC_NEUMANN))
    return PIC_ERR_ARG;
  if (c->bc_lo == PIC_BC_NEUMANN && c->bc_hi == PIC_BC_NEUMANN)
    return PIC_ERR_ARG;
  if (c->precision != PIC_FP64 && c->precision != PIC_MIXED) return PIC_ERR_ARG;
  if (!(c->rel_tol > 0.0) || c->max_vcycles < 1 || c->nu_pre < 0 ||
      c->nu_post < 0 || c->nu_pre + c->nu_post < 1 || c->coarse_sweeps < 1)
    return PIC_ERR_ARG;
  if (c->sort_every != 1) return PIC_ERR_ARG;
  if (c->w_sp < 1) return PIC_ERR_ARG;
  for (int s = 0; s < PIC_NSPECIES; ++s)
    if (c->capacity[s] < 0 || c->capacity[s] > 0xFFFFFFF0ll) return PIC_ERR_ARG;
  if (c->queue_capacity < 0 || c->max_events < 1) return PIC_ERR_ARG;
  const long long nodes = (long long)c->nx * c->ny * (c->nz + 1);
  if (nodes > 0x7FFFFFFFll) return PIC_ERR_ARG;
  // Cell records keep the (tile-major) cell number above two species bits.
  if ((c->flags & PIC_FLAG_CELL_GROUPS) &&
      (long long)((c->nx + 7) / 8) * ((c->ny + 7) / 8) * ((c->nz + 7) / 8) * 512 >=
          (1ll << 30))
    return PIC_ERR_ARG;
  // Their counts, offsets and index words (a particle's position in the
  // three species taken together) are 32-bit.
  if ((c->flags & PIC_FLAG_CELL_GROUPS) &&
      c->capacity[0] + c->capacity[1] + c->capacity[2] > 0xFFFFFFF0ll)
    return PIC_ERR_ARG;
  return PIC_OK;
}

// Lay out every device array of a context in the workspace (base == nullptr:
// size only).
size_t carve(pic_ctx* c, char* base) {
  Carver cv{base, 0};
  const pic_config& f = c->cfg;
  const bool mixed = f.precision == PIC_MIXED;
  for (int s = 0; s < PIC_NSPECIES; ++s) {
    const long long cap = f.capacity[s];
    for (int b = 0; b < 2; ++b) {
      if (!mixed) {
        Parts& p = c->P[s][b];
        p.x = cv.take<double>(cap); p.y = cv.take<double>(cap);
        p.z = cv.take<double>(cap); p.vx = cv.take<double>(cap);
        p.vy = cv.take<double>(cap); p.vz = cv.take<double>(cap);
        p.id = cv.take<uint64_t>(cap);
      } else {
        PartsM& p = c->PM[s][b];
        p.cell = cv.take<uint32_t>(cap);
        p.ox = cv.take<float>(cap); p.oy = cv.take<float>(cap);
        p.oz = cv.take<float>(cap); p.vx = cv.take<float>(cap);
        p.vy = cv.take<float>(cap); p.vz = cv.take<float>(cap);
        p.id = cv.take<uint64_t>(cap);
      }
    }
    c->key[s] = cv.take<uint32_t>(cap);
    c->tsb[s][0] = cv.take<uint32_t>(c->ntiles + 1);
    c->tsb[s][1] = cv.take<uint32_t>(c->ntiles + 1);
  }
  c->tile_cursor = cv.take<uint32_t>(c->ntiles + 1);
  c->tcnt[0] = cv.take<uint32_t>(2 * (c->ntiles + 1));
  c->tcnt[1] = c->tcnt[0] + (c->ntiles + 1);
  const long long nsb = (c->ntiles + 1 + 1023) / 1024;
  c->scan_block = cv.take<uint32_t>(2 * nsb + 2);
  c->acc = cv.take<long long>(c->nnodes);
  c->acc_next = cv.take<long long>(c->nnodes);
  c->E = reinterpret_cast<double*>(
      cv.take<char>(3 * c->nnodes * (long long)(mixed ? 4 : 8)));
  for (int l = 0; l < c->nlev; ++l) {
    Level& L = c->lev[l];
    L.u = L.f = L.us = nullptr;
    L.uf = L.ff = L.usf = nullptr;
    if (l == 0 || !mixed) {
      L.u = cv.take<double>(L.nnodes);
      L.f = cv.take<double>(L.nnodes);
      if (!mixed) L.us = cv.take<double>(L.nnodes);
    }
    if (mixed) {
      L.uf = cv.take<float>(L.nnodes);
      L.ff = cv.take<float>(L.nnodes);
      L.usf = cv.take<float>(L.nnodes);
    }
  }
  c->partials = cv.take<double>(c->npartials);
  {
    const long long es = mixed ? 4 : 8;
    const long long pm = (long long)c->spec_planes * c->spec_modes;
    c->spec_s = cv.take<char>(2 * pm * es);
    c->spec_m = cv.take<char>(pm * es);
  }
  c->part_n = cv.take<double>(neutral_push_blocks(f.capacity[1]));
  c->qpartials = cv.take<long long>(1024);
  c->ncount = cv.take<int>(c->ncells);
  c->flag = cv.take<uint32_t>((c->ncells + 31) / 32);
  c->cand = cv.take<CandRec>(f.capacity[0]);
  c->dead1 = cv.take<uint32_t>(kDeadList);
  c->dead2 = cv.take<uint32_t>(kDeadList);
  c->rm_pairs = cv.take<uint2>(kDeadList);
  c->cand_cnt = cv.take<uint32_t>(c->nch_cap + 1);
  c->el_cnt = cv.take<uint32_t>(c->nch_cap + 1);
  c->chunks = cv.take<uint2>(c->nch_cap);
  c->cstart = cv.take<uint32_t>(c->ntiles + 1);
  c->cmp_idx = cv.take<uint32_t>(2 * f.capacity[1]);
  c->ev = cv.take<Rec>(c->ev_cap_p2);
  c->nc = cv.take<Rec>(c->ev_cap_p2);
  c->ok = cv.take<Rec>(c->ev_cap_p2);
  c->okp = cv.take<uint2>(c->ev_cap_p2);
  c->rec_tmp = cv.take<Rec>(c->ev_cap_p2);
  c->ab_rec = cv.take<Rec>(c->ev_cap_p2);
  c->ab_raw_pos = cv.take<double>(3 * f.max_events);
  c->ab_raw_vel = cv.take<double>(3 * f.max_events);
  c->ab_species = cv.take<int32_t>(f.max_events);
  c->ab_id = cv.take<uint64_t>(f.max_events);
  c->ab_pos = cv.take<double>(3 * f.max_events);
  c->ab_vel = cv.take<double>(3 * f.max_events);
  c->q_pos = cv.take<double>(3 * f.queue_capacity);
  c->q_vel = cv.take<double>(3 * f.queue_capacity);
  c->fn_scan = cv.take<unsigned>(2 * c->g.nxy + 2);
  c->dc = cv.take<Counters>(1);
  c->cg_cnt = c->cg_off = c->cg_bsum = c->cg_big = c->cg_nbig = nullptr;
  c->cg_rec = c->cg_srt = nullptr;
  c->cg_idx = c->cg_poff = c->cg_hot = c->cg_hpre = c->cg_rest = nullptr;
  c->cg_work_cap = 0;
  c->ip_ev = nullptr;
  c->ip_evp = nullptr;
  c->cg_big_cap = 0;
  c->cg_nkeys = c->ntiles * kTile * kTile * kTile;
  if (f.flags & PIC_FLAG_CELL_GROUPS) {
    c->cg_cnt = cv.take<unsigned>(c->cg_nkeys);
    c->cg_off = cv.take<unsigned>(c->cg_nkeys + 1);
    c->cg_bsum = cv.take<unsigned>(coulomb_scan_blocks(c->cg_nkeys));
    c->cg_big_cap = std::min<long long>(c->ncells, 1ll << 16);
    c->cg_big = cv.take<unsigned>(c->cg_big_cap);
    c->cg_nbig = cv.take<unsigned>(4);
    c->cg_work_cap = f.capacity[0] + f.capacity[1] + f.capacity[2];
    c->cg_rec = cv.take<Rec>(c->cg_work_cap);
    c->cg_srt = cv.take<Rec>(c->cg_work_cap);
    c->cg_idx = cv.take<unsigned>(c->cg_work_cap);
    // One tile plane: kTile x kTile cells.
    c->cg_poff = cv.take<unsigned>(c->cg_nkeys / (kTile * kTile) + 1);
    c->cg_hot = cv.take<unsigned>(c->cg_nkeys / (kTile * kTile));
    c->cg_hpre = cv.take<unsigned>(c->cg_nkeys / (kTile * kTile) + 1);
    c->cg_rest = cv.take<unsigned>(c->cg_nkeys / (kTile * kTile));
    c->ip_ev = cv.take<Rec>(c->ev_cap_p2);
    c->ip_evp = cv.take<uint2>(c->ev_cap_p2);
  }
  c->dbg_mom = cv.take<double>(debye_moment_doubles(c->ncells));
  c->dbg_qpart = cv.take<long long>(2048);
  c->dbg_part = cv.take<double>(2048);
  c->dbg_out = cv.take<double>(4);
  c->warm_x = cv.take<float>(2 * c->g.nxy * f.nz);
  c->warm_prev = cv.take<double>(c->nnodes);
  c->phi_hist = cv.take<double>(c->nnodes);
  return cv.off + kAlign;
}

// The arrays the field solve alone uses (allocation-free poisson solve):
// the multigrid levels, the reduction partials, the exact coarse level and
// the counters.
size_t carve_field(pic_ctx* c, char* base) {
  Carver cv{base, 0};
  const bool mixed = c->cfg.precision == PIC_MIXED;
  for (int l = 0; l < c->nlev; ++l) {
    Level& L = c->lev[l];
    L.u = L.f = L.us = nullptr;
    L.uf = L.ff = L.usf = nullptr;
    if (l == 0 || !mixed) {
      L.u = cv.take<double>(L.nnodes);
      L.f = cv.take<double>(L.nnodes);
      if (!mixed) L.us = cv.take<double>(L.nnodes);
    }
    if (mixed) {
      L.uf = cv.take<float>(L.nnodes);
      L.ff = cv.take<float>(L.nnodes);
      L.usf = cv.take<float>(L.nnodes);
    }
  }
  c->partials = cv.take<double>(c->npartials);
  {
    const long long es = mixed ? 4 : 8;
    const long long pm = (long long)c->spec_planes * c->spec_modes;
    c->spec_s = cv.take<char>(2 * pm * es);
    c->spec_m = cv.take<char>(pm * es);
  }
  c->qpartials = cv.take<long long>(1024);
  c->dc = cv.take<Counters>(1);
  return cv.off + kAlign;
}

void derive(pic_ctx* c) {
  const pic_config& f = c->cfg;
  c->mixed = f.precision == PIC_MIXED;
  GridC& g = c->g;
  g.nx = f.nx; g.ny = f.ny; g.nz = f.nz;
  g.tnx = (f.nx + kTile - 1) / kTile;
  g.tny = (f.ny + kTile - 1) / kTile;
  g.tnz = (f.nz + kTile - 1) / kTile;
  g.dx = f.dx;
  g.inv_dx = 1.0 / f.dx;
  g.lx = (double)f.nx * f.dx;
  g.ly = (double)f.ny * f.dx;
  g.nxy = (long long)f.nx * f.ny;
  c->nnodes = g.nxy * (f.nz + 1);
  c->ncells = g.nxy * f.nz;
  c->ntiles = (long long)g.tnx * g.tny * g.tnz;
  int dims[16][3];
  c->nlev = plan_levels(&f, dims);
  double h2 = 1.0;
  for (int l = 0; l < c->nlev; ++l) {
    Level& L = c->lev[l];
    L.nx = dims[l][0]; L.ny = dims[l][1]; L.nz = dims[l][2];
    L.nnodes = (long long)L.nx * L.ny * (L.nz + 1);
    L.h2 = h2;
    h2 *= 4.0;
  }
  // The first coarse level small enough for the exact solve.
  c->spec_level = -1;
  c->spec_modes = c->spec_planes = 0;
  if (!(f.flags & PIC_FLAG_MG_ALL_LEVELS)) {
    for (int l = 1; l < c->nlev; ++l) {
      const Level& L = c->lev[l];
      const int k0 = f.bc_lo == PIC_BC_DIRICHLET ? 1 : 0;
      const int k1 = f.bc_hi == PIC_BC_DIRICHLET ? L.nz - 1 : L.nz;
      auto pow2 = [](int n) { return n > 0 && !(n & (n - 1)); };
      const bool by_fft = pow2(L.nx) && pow2(L.ny) && L.nx <= kSpecMaxFFT &&
                          L.ny <= kSpecMaxFFT;
      const bool direct = L.nx <= kSpecMaxXY && L.ny <= kSpecMaxXY;
      if (L.nx >= 2 && L.ny >= 2 && !(L.nx & 1) && !(L.ny & 1) &&
          (by_fft || direct) && k1 >= k0 && k1 - k0 + 1 <= kSpecMaxPlanes) {
        c->spec_level = l;
        c->spec_modes = L.ny * (L.nx / 2 + 1);
        c->spec_planes = k1 - k0 + 1;
        break;
      }
    }
  }
  long long maxcap = std::max(std::max(f.capacity[0], f.capacity[3]),
                              std::max(f.capacity[1], f.capacity[2]));
  // Chunk list of the charged species: at most one chunk per tile plus one
  // per 2048 particles.
  c->nch_cap = c->ntiles + (f.capacity[0] + f.capacity[2]) / 2048 + 4;
  c->npartials = (int)(2 * c->nch_cap + 3 * (maxcap / 256 + 64) + 4096 +
                       2ll * (f.nz + 2));
  c->ev_cap_p2 = pow2_at_least(std::max<long long>(f.max_events, 2));
}

pic_status sync_counters(pic_ctx* c) {
  if (!hip_ok(c, hipMemcpyAsync(c->hpin, c->dc, sizeof(Counters),
                                hipMemcpyDeviceToHost, c->stream),
              "counter readback"))
    return PIC_ERR_HIP;
  if (!hip_ok(c, stream_wait(c), "stream synchronise")) return PIC_ERR_HIP;
  c->hc = *c->hpin;
  return PIC_OK;
}

pic_status check_flags(pic_ctx* c) {
  const unsigned e = c->hc.err;
  if (!e) return PIC_OK;
  hipMemsetAsync(&c->dc->err, 0, sizeof(unsigned), c->stream);
  if (e & kErrNonFinite)
    return set_err(c, PIC_ERR_NONFINITE, "non-finite or out-of-domain value");
  if (e & kErrCapacity)
    return set_err(c, PIC_ERR_CAPACITY, "particle capacity exceeded");
  if (e & kErrEvents)
    return set_err(c, PIC_ERR_CAPACITY,
                   "per-step event list (max_events) exceeded");
  return set_err(c, PIC_ERR_STATE, "device error flag");
}

__global__ void k_set_n(Counters* dc, int s, unsigned long long n) {
  dc->n[s] = n;
}

__global__ void k_deinterleave_E(const char* __restrict__ E, int mixed,
                                 double* __restrict__ out, long long n) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  for (int d = 0; d < 3; ++d) {
    out[d * n + t] = mixed ? (double)reinterpret_cast<const float*>(E)[d * n + t]
                           : reinterpret_cast<const double*>(E)[d * n + t];
  }
}

// Accumulate the elapsed time of every phase recorded since the last
// collection (the stream has been synchronised).
void collect_times(pic_ctx* c) {
  if (!c->timing) return;
  for (int p = 0; p < PIC_NPHASES; ++p) {
    for (int i = 0; i < c->tn[p]; ++i) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, c->tev[p][i][0], c->tev[p][i][1]) ==
          hipSuccess) {
        c->tms[p] += ms;
        c->tcalls[p] += 1;
      }
    }
    c->tn[p] = 0;
  }
}

void fill_diag(pic_ctx* c, pic_diag* d) {
  if (!d) return;
  const Counters& h = c->hc;
  for (int s = 0; s < PIC_NSPECIES; ++s) {
    d->counts[s] = c->n[s];
    d->cathode[s] = (long long)h.cathode[s];
    d->anode[s] = (long long)h.anode[s];
    d->kinetic[s] = h.kinetic[s];
  }
  d->fn_emitted = (long long)h.fn_total;
  d->candidates = (long long)h.n_cand;
  d->elastic = (long long)h.n_elastic;
  d->ionisations = (long long)h.n_ok;
  d->starved = (long long)h.n_events - (long long)h.n_ok;
  d->over_majorant = (long long)h.n_over;
  d->near_threshold = (long long)h.n_near;
  d->total_charge_units = h.total_charge;
  d->field_energy = h.field_energy;
  d->np_absorbed = (long long)h.np_hits;
  d->np_heat = h.np_heat;
  d->coulomb_like = (long long)h.coul_like;
  d->coulomb_ei = (long long)h.coul_ei;
  d->recombinations = (long long)h.f3_rec;
  d->ionisations2 = (long long)h.f3_ion2;
  d->charge_exchanges = (long long)h.f3_cx;
  d->ion_starved = (long long)h.f3_starved;
  d->solve = c->last_solve;
  d->step = c->step;
  d->next_id = c->next_id;
}

}  // namespace

extern "C" {

int32_t pic_abi_version(void) { return PIC_ABI_VERSION; }

const char* pic_last_error(const pic_ctx* c) {
  return c ? c->err.c_str() : "null context";
}

pic_status pic_workspace_bytes(const pic_config* cfg, size_t* bytes) {
  if (!bytes) return PIC_ERR_ARG;
  const pic_status v = validate(cfg);
  if (v != PIC_OK) return v;
  pic_ctx* c = new (std::nothrow) pic_ctx();
  if (!c) return PIC_ERR_STATE;
  c->cfg = *cfg;
  derive(c);
  *bytes = carve(c, nullptr);
  delete c;
  return PIC_OK;
}

pic_status pic_init(const pic_config* cfg, void* ws, size_t bytes,
                    void* stream, pic_ctx** out) {
  if (!out) return PIC_ERR_ARG;
  *out = nullptr;
  const pic_status v = validate(cfg);
  if (v != PIC_OK) return v;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign)) return PIC_ERR_ARG;
  pic_ctx* c = new (std::nothrow) pic_ctx();
  if (!c) return PIC_ERR_STATE;
  c->cfg = *cfg;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  derive(c);
  const size_t need = carve(c, nullptr);
  if (bytes < need) {
    delete c;
    return PIC_ERR_ARG;
  }
  char* base = reinterpret_cast<char*>(
      (reinterpret_cast<uintptr_t>(ws) + kAlign - 1) / kAlign * kAlign);
  c->ws = reinterpret_cast<char*>(ws);
  c->ws_bytes = bytes;
  carve(c, base);
  for (int s = 0; s < PIC_NSPECIES; ++s) {
    c->cur[s] = 0;
    c->tcur[s] = 0;
    c->n[s] = 0;
    c->n_binned[s] = 0;
  }
  c->nch_bound = 1;
  c->tcounted = false;
  c->ncount_valid = false;
  c->acc_next_valid = false;
  c->n_start1 = 0;
  c->ion_moved_accum = 0;
  c->ions_binned = true;
  c->hmid = nullptr;
  c->ev_mid = nullptr;
  c->hpin = nullptr;
  c->ev_sync = nullptr;
  c->next_id = 0;
  c->step = 0;
  c->queue_used = 0;
  c->last_vcycles = 0;
  c->warm_mode = PIC_WS_PREV;
  c->spec_ready = false;
  c->u_solved = false;
  c->hist_valid = false;
  c->net = nullptr;
  c->warm_recorded = false;
  std::memset(&c->coll, 0, sizeof(c->coll));
  std::memset(&c->coul, 0, sizeof(c->coul));
  std::memset(&c->ionp, 0, sizeof(c->ionp));
  std::memset(&c->src, 0, sizeof(c->src));
  std::memset(&c->last_solve, 0, sizeof(c->last_solve));
  std::memset(&c->hc, 0, sizeof(c->hc));
  c->timing = false;
  c->ev_made = false;
  if (!hip_ok(c, hipMemsetAsync(ws, 0, bytes, c->stream), "workspace clear") ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "init synchronise") ||
      !hip_ok(c, hipHostMalloc(reinterpret_cast<void**>(&c->hmid), sizeof(Counters),
                               hipHostMallocDefault),
              "pinned counters") ||
      !hip_ok(c, hipHostMalloc(reinterpret_cast<void**>(&c->hpin), sizeof(Counters),
                               hipHostMallocDefault),
              "pinned counters") ||
      !hip_ok(c, hipEventCreateWithFlags(&c->ev_mid, hipEventDisableTiming),
              "event create") ||
      !hip_ok(c, hipEventCreateWithFlags(&c->ev_sync, hipEventDisableTiming),
              "event create")) {
    if (c->hmid) hipHostFree(c->hmid);
    if (c->hpin) hipHostFree(c->hpin);
    if (c->ev_mid) hipEventDestroy(c->ev_mid);
    if (c->ev_sync) hipEventDestroy(c->ev_sync);
    delete c;
    return PIC_ERR_HIP;
  }
  *out = c;
  return PIC_OK;
}

void pic_destroy(pic_ctx* c) {
  if (!c) return;
  if (c->hmid) hipHostFree(c->hmid);
  if (c->hpin) hipHostFree(c->hpin);
  if (c->ev_mid) hipEventDestroy(c->ev_mid);
  if (c->ev_sync) hipEventDestroy(c->ev_sync);
  if (c->ev_made)
    for (int p = 0; p < PIC_NPHASES; ++p)
      for (int i = 0; i < pic_ctx::kTimeIv; ++i)
        for (int e = 0; e < 2; ++e) hipEventDestroy(c->tev[p][i][e]);
  delete c;
}

pic_status pic_enable_timing(pic_ctx* c, int32_t on) {
  if (!c) return PIC_ERR_ARG;
  if (on && !c->ev_made) {
    for (int p = 0; p < PIC_NPHASES; ++p)
      for (int i = 0; i < pic_ctx::kTimeIv; ++i)
        for (int e = 0; e < 2; ++e)
          if (!hip_ok(c, hipEventCreate(&c->tev[p][i][e]), "event create"))
            return PIC_ERR_HIP;
    c->ev_made = true;
  }
  c->timing = on != 0;
  for (int p = 0; p < PIC_NPHASES; ++p) {
    c->tms[p] = 0.0;
    c->tcalls[p] = 0;
    c->tn[p] = 0;
  }
  return PIC_OK;
}

pic_status pic_phase_times(pic_ctx* c, double* ms, int64_t* calls) {
  if (!c || !ms) return PIC_ERR_ARG;
  for (int p = 0; p < PIC_NPHASES; ++p) {
    ms[p] = c->tms[p];
    if (calls) calls[p] = c->tcalls[p];
  }
  return PIC_OK;
}

pic_status pic_set_collisions(pic_ctx* c, const pic_collisions* k) {
  if (!c || !k) return PIC_ERR_ARG;
  if (k->enabled) {
    if (k->ion_model != PIC_ION_LOTZ && k->ion_model != PIC_ION_CONST)
      return set_err(c, PIC_ERR_ARG, "unknown ionisation model");
    if (!(k->sigma_el >= 0.0) || !(k->lotz_a >= 0.0) || !(k->ion_I_eV > 0.0) ||
        !(k->sigma_ion_const >= 0.0) || !(k->E_max_eV > 0.0))
      return set_err(c, PIC_ERR_ARG, "invalid collision parameters");
  }
  c->coll = *k;
  return PIC_OK;
}

pic_status pic_set_coulomb(pic_ctx* c, const pic_coulomb* k) {
  if (!c || !k) return PIC_ERR_ARG;
  if (k->enabled) {
    if (!c->cg_rec)
      return set_err(c, PIC_ERR_STATE,
                     "Coulomb collisions need PIC_FLAG_CELL_GROUPS at init");
    if (!(k->ln_lambda > 0.0) || !std::isfinite(k->ln_lambda))
      return set_err(c, PIC_ERR_ARG, "invalid Coulomb logarithm");
  }
  c->coul = *k;
  return PIC_OK;
}

pic_status pic_set_ion_processes(pic_ctx* c, const pic_ion_processes* k) {
  if (!c || !k) return PIC_ERR_ARG;
  if (k->enabled) {
    if (!c->cg_rec)
      return set_err(c, PIC_ERR_STATE,
                     "ion processes need PIC_FLAG_CELL_GROUPS at init");
    if (!(k->sigma_rec_1eV >= 0.0) || !(k->lotz_a2 >= 0.0) ||
        !(k->ion2_I_eV > 0.0) || !std::isfinite(k->cx_a) ||
        !std::isfinite(k->cx_b) || !std::isfinite(k->sigma_rec_1eV))
      return set_err(c, PIC_ERR_ARG, "invalid ion-process parameters");
  }
  c->ionp = *k;
  return PIC_OK;
}

pic_status pic_set_sources(pic_ctx* c, const pic_sources* s) {
  if (!c || !s) return PIC_ERR_ARG;
  const double lx = c->g.lx, ly = c->g.ly, lmin = std::min(lx, ly);
  const double lz = (double)c->g.nz * c->g.dx;
  auto in_xy = [&](double x, double y) {
    return x >= 0.0 && x < lx && y >= 0.0 && y < ly;
  };
  // Source particles must start inside the domain: centres inside, radii
  // below one period (one wrap suffices), the sphere clear of both faces.
  if ((s->disk_on && (s->disk_n_e < 0 || s->disk_n_n < 0 ||
                      !(s->disk_radius >= 0.0) || !(s->disk_radius < lmin) ||
                      !in_xy(s->disk_cx, s->disk_cy))) ||
      (s->sphere_on &&
       (s->sph_n < 0 || !(s->sph_radius >= 0.0) || !(s->sph_radius < lmin) ||
        !in_xy(s->sph_cx, s->sph_cy) || !(s->sph_cz - s->sph_radius >= 0.0) ||
        !((s->sph_cz + s->sph_radius) * c->g.inv_dx < (double)c->g.nz))) ||
      (s->fn_on && !(s->fn_phi_w_eV > 0.0)) ||
      (s->sph_absorb &&
       (!(s->sph_radius > 0.0) || !(s->sph_radius < 0.5 * lmin) ||
        !in_xy(s->sph_cx, s->sph_cy) || !(s->sph_cz - s->sph_radius >= 0.0) ||
        !((s->sph_cz + s->sph_radius) * c->g.inv_dx < (double)c->g.nz) ||
        !(s->sph_alpha_eh >= 0.0 && s->sph_alpha_eh <= 1.0))))
    return set_err(c, PIC_ERR_ARG, "invalid source parameters");
  (void)lz;
  c->src = *s;
  return PIC_OK;
}

pic_status pic_inject(pic_ctx* c, int32_t species, int64_t n,
                      const double* pos, const double* vel) {
  if (!c || species < 0 || species >= PIC_NSPECIES || n < 0) return PIC_ERR_ARG;
  if (n == 0) return PIC_OK;
  if (!pos || !vel) return set_err(c, PIC_ERR_ARG, "null particle buffer");
  if (c->queue_used + n > c->cfg.queue_capacity)
    return set_err(c, PIC_ERR_CAPACITY, "injection queue full");
  if (!parts_validate(c, pos, vel, n))
    return set_err(c, PIC_ERR_ARG,
                   "injected particle outside the domain or non-finite");
  const long long off = c->queue_used;
  // The queue keeps each call's SoA block contiguous: 3n values per array.
  if (!hip_ok(c, hipMemcpyAsync(c->q_pos + 3 * off, pos, 3 * n * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream),
              "inject copy") ||
      !hip_ok(c, hipMemcpyAsync(c->q_vel + 3 * off, vel, 3 * n * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream),
              "inject copy"))
    return PIC_ERR_HIP;
  c->queue.push_back(QueueCall{species, n, off});
  c->queue_used += n;
  return PIC_OK;
}

pic_status pic_deposit(pic_ctx* c) {
  if (!c) return PIC_ERR_ARG;
  parts_deposit(c);
  return hip_ok(c, hipGetLastError(), "deposit launch") ? PIC_OK : PIC_ERR_HIP;
}

pic_status pic_field(pic_ctx* c, pic_solve_info* info) {
  if (!c) return PIC_ERR_ARG;
  const bool extrap = c->warm_mode == PIC_WS_EXTRAP;
  if (extrap) {
    tmark(c, PIC_PH_WARM, true);
    field_extrapolate(c);
    tmark(c, PIC_PH_WARM, false);
  }
  tmark(c, PIC_PH_RHS, true);
  field_rhs(c, nullptr);
  tmark(c, PIC_PH_RHS, false);
  int st = PIC_OK;
  pic_solve_info loc;
  tmark(c, PIC_PH_POISSON, true);
  field_solve(c, true, &loc, &st);
  tmark(c, PIC_PH_POISSON, false);
  c->last_solve = loc;
  // The next extrapolation needs this solve and the one before it.
  c->hist_valid = extrap && c->u_solved && st == PIC_OK;
  c->u_solved = st == PIC_OK;
  if (info) *info = loc;
  tmark(c, PIC_PH_EFIELD, true);
  field_efield(c);
  tmark(c, PIC_PH_EFIELD, false);
  if (!hip_ok(c, hipGetLastError(), "field launch")) return PIC_ERR_HIP;
  if (st != PIC_OK)
    return set_err(c, (pic_status)st, "Poisson solve did not converge");
  return PIC_OK;
}

pic_status pic_set_phi(pic_ctx* c, const double* phi) {
  if (!c || !phi) return PIC_ERR_ARG;
  c->u_solved = c->hist_valid = false;
  if (!hip_ok(c, hipMemcpyAsync(c->lev[0].u, phi, c->nnodes * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream),
              "phi copy"))
    return PIC_ERR_HIP;
  field_efield(c);
  return hip_ok(c, hipGetLastError(), "efield launch") ? PIC_OK : PIC_ERR_HIP;
}

namespace {

// Host-known additions of the next step (queue, disk, sphere) must fit.
pic_status advance_check(pic_ctx* c, double dt, long long add[PIC_NSPECIES]) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_err(c, PIC_ERR_ARG, "dt");
  for (int k = 0; k < PIC_NSPECIES; ++k) add[k] = 0;
  for (const QueueCall& q : c->queue) add[q.species] += q.n;
  const pic_sources& s = c->src;
  if (s.disk_on) {
    add[0] += s.disk_n_e;
    add[1] += s.disk_n_n;
  }
  if (s.sphere_on) add[1] += s.sph_n;
  for (int k = 0; k < PIC_NSPECIES; ++k)
    if (c->n[k] + add[k] > c->cfg.capacity[k])
      return set_err(c, PIC_ERR_CAPACITY, "sources exceed particle capacity");
  return PIC_OK;
}

// The field-dependent rest of a step (after the host-known sources and the
// neutral push), the binning pass, the synchronisation and the host
// bookkeeping.
pic_status advance_finish(pic_ctx* c, double dt,
                          const long long add[PIC_NSPECIES],
                          pic_absorbed* out, pic_diag* diag) {
  parts_sources_fn(c, dt);
  parts_push_collide(c, dt);
  parts_bin(c);
  if (!hip_ok(c, hipGetLastError(), "advance launch")) return PIC_ERR_HIP;
  pic_status st = sync_counters(c);
  if (st != PIC_OK) return st;
  for (int k = 0; k < PIC_NSPECIES; ++k) {
    if (k == 2 && !c->ions_binned) {
      c->n[k] = (long long)c->hc.n[k];   // binned ranges kept, tail grown
      continue;
    }
    c->n[k] = (long long)c->hc.sorted_n[k];
    c->n_binned[k] = c->n[k];
  }
  c->next_id = c->hc.next_id;
  c->step += 1;
  collect_times(c);
  if (diag) {
    fill_diag(c, diag);
    for (int k = 0; k < PIC_NSPECIES; ++k) diag->emitted[k] = add[k];
    diag->emitted[0] += (long long)c->hc.fn_total;
  }
  if (out) {
    long long n = (long long)c->hc.n_ab;
    if (n > c->cfg.max_events) n = c->cfg.max_events;
    out->n = n;
    out->species = c->ab_species;
    out->id = c->ab_id;
    out->pos = c->ab_pos;
    out->vel = c->ab_vel;
  }
  return check_flags(c);
}

}  // namespace

pic_status pic_advance(pic_ctx* c, double dt, pic_absorbed* out,
                       pic_diag* diag) {
  if (!c) return PIC_ERR_ARG;
  long long add[PIC_NSPECIES];
  const pic_status v = advance_check(c, dt, add);
  if (v != PIC_OK) return v;
  parts_sources_host(c);
  parts_push_neutral(c, dt);
  const pic_status st = advance_finish(c, dt, add, out, diag);
  // After a failed step the neutrals are counted and the charge deposited
  // afresh.
  c->acc_next_valid = st == PIC_OK;
  if (st != PIC_OK) c->ncount_valid = false;
  return st;
}

pic_status pic_step(pic_ctx* c, double dt, pic_absorbed* out, pic_diag* diag) {
  if (!c) return PIC_ERR_ARG;
  pic_status st = pic_deposit(c);
  if (st != PIC_OK) return st;
  st = pic_field(c, nullptr);
  if (st != PIC_OK) return st;
  return pic_advance(c, dt, out, diag);
}

pic_status poisson_solve(pic_ctx* c, const double* rho, double* phi,
                         int32_t warm, pic_solve_info* info) {
  if (!c || !rho || !phi) return PIC_ERR_ARG;
  c->u_solved = c->hist_valid = false;
  if (warm == PIC_WARM_GIVEN) {
    if (!hip_ok(c, hipMemcpyAsync(c->lev[0].u, phi, c->nnodes * sizeof(double),
                                  hipMemcpyDeviceToDevice, c->stream),
                "phi copy"))
      return PIC_ERR_HIP;
  }
  field_rhs(c, rho);
  int st = PIC_OK;
  pic_solve_info loc;
  field_solve(c, warm == PIC_WARM_GIVEN, &loc, &st);
  if (info) *info = loc;
  if (!hip_ok(c, hipMemcpyAsync(phi, c->lev[0].u, c->nnodes * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream),
              "phi copy") ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "synchronise"))
    return PIC_ERR_HIP;
  if (st != PIC_OK)
    return set_err(c, (pic_status)st, "Poisson solve did not converge");
  return PIC_OK;
}

// ---- allocation-free Poisson solve ------------------------------------------
}  // extern "C"

// The fixed device buffer of poisson_solve_static: one per GPU the library
// runs on, held until the process ends.  Host code never passes the array's
// name to a kernel or a copy (on the host it is only a stand-in for the
// symbol): it uses the device address hipGetSymbolAddress returns, looked up
// once per device.
static __device__ __align__(256) char scratch[PIC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};
// Counter readbacks of the allocation-free solve land here (pageable host
// memory, one slot per device).
Counters g_scratch_counters[kMaxDevices];

__global__ void k_zero16(uint4* __restrict__ p, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

extern "C" {

pic_status poisson_solve_static(const pic_config* cfg, const double* rho,
                                double* phi, int32_t warm,
                                pic_solve_info* info, void* stream) {
  if (!cfg || !rho || !phi) return PIC_ERR_ARG;
  if (warm != PIC_WARM_ZERO && warm != PIC_WARM_GIVEN) return PIC_ERR_ARG;
  if (validate(cfg) != PIC_OK) return PIC_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return PIC_ERR_HIP;
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
        return PIC_ERR_HIP;
      g_scratch_ptr[dev] = static_cast<char*>(ptr);
    }
    base = g_scratch_ptr[dev];
  }
  // A field-only context on the stack: the particle capacities are zero and
  // every device array comes from the fixed buffer.
  pic_ctx c{};
  c.cfg = *cfg;
  for (int s = 0; s < PIC_NSPECIES; ++s) c.cfg.capacity[s] = 0;
  c.cfg.queue_capacity = 0;
  c.cfg.max_events = 1;
  c.stream = reinterpret_cast<hipStream_t>(stream);
  derive(&c);
  const size_t need = carve_field(&c, nullptr);
  if (need > (size_t)PIC_STATIC_SCRATCH_BYTES) return PIC_ERR_CAPACITY;
  carve_field(&c, base);
  c.hpin = &g_scratch_counters[dev];
  c.ev_sync = nullptr;
  c.warm_mode = PIC_WS_PREV;
  c.last_vcycles = 0;
  c.spec_ready = false;
  c.timing = false;
  // Every array starts at zero, whatever the last call on this GPU left.
  const long long n16 = (long long)(need / 16);
  k_zero16<<<1024, 256, 0, c.stream>>>(reinterpret_cast<uint4*>(base), n16);
  if (hipGetLastError() != hipSuccess) return PIC_ERR_HIP;
  if (warm == PIC_WARM_GIVEN &&
      hipMemcpyAsync(c.lev[0].u, phi, c.nnodes * sizeof(double),
                     hipMemcpyDeviceToDevice, c.stream) != hipSuccess)
    return PIC_ERR_HIP;
  field_rhs(&c, rho);
  int st = PIC_OK;
  pic_solve_info loc;
  field_solve(&c, warm == PIC_WARM_GIVEN, &loc, &st);
  if (info) *info = loc;
  if (hipMemcpyAsync(phi, c.lev[0].u, c.nnodes * sizeof(double),
                     hipMemcpyDeviceToDevice, c.stream) != hipSuccess ||
      hipStreamSynchronize(c.stream) != hipSuccess)
    return PIC_ERR_HIP;
  return (pic_status)st;
}

pic_status pic_set_warm_start(pic_ctx* c, int32_t mode, pic_unet* net) {
  if (!c) return PIC_ERR_ARG;
  if (mode != PIC_WS_PREV && mode != PIC_WS_RECORD && mode != PIC_WS_UNET &&
      mode != PIC_WS_EXTRAP)
    return set_err(c, PIC_ERR_ARG, "unknown warm-start mode");
  if (mode == PIC_WS_UNET) {
    if (!net) return set_err(c, PIC_ERR_ARG, "learned warm start needs a network");
    const pic_config& f = c->cfg;
    if ((f.nx & 7) || (f.ny & 7) || (f.nz & 7) || f.nx < 8 || f.ny < 8 ||
        f.nz < 8 || !pic_unet_fits(net, f.nz, f.ny, f.nx))
      return set_err(c, PIC_ERR_ARG,
                     "grid (nz, ny, nx) must be multiples of 8 within the network's size");
  }
  c->warm_mode = mode;
  c->net = mode == PIC_WS_UNET ? net : nullptr;
  c->warm_recorded = false;
  return PIC_OK;
}

pic_status pic_warm_pair(pic_ctx* c, float* input, float* target) {
  if (!c || (!input && !target)) return PIC_ERR_ARG;
  if (!c->warm_recorded)
    return set_err(c, PIC_ERR_STATE, "no solve has recorded a warm-start pair");
  if (input &&
      !hip_ok(c, hipMemcpyAsync(input, c->warm_x,
                                2 * c->g.nxy * c->cfg.nz * sizeof(float),
                                hipMemcpyDeviceToDevice, c->stream),
              "pair copy"))
    return PIC_ERR_HIP;
  if (target) field_warm_target(c, target);
  if (!hip_ok(c, hipGetLastError(), "pair launch") ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "synchronise"))
    return PIC_ERR_HIP;
  return PIC_OK;
}

pic_status pic_load_particles(pic_ctx* c, int32_t s, int64_t n,
                              const double* pos, const double* vel,
                              const uint64_t* ids) {
  if (!c || s < 0 || s >= PIC_NSPECIES || n < 0) return PIC_ERR_ARG;
  if (n > c->cfg.capacity[s])
    return set_err(c, PIC_ERR_CAPACITY, "load exceeds capacity");
  if (n > 0 && (!pos || !vel || !ids)) return PIC_ERR_ARG;
  parts_load(c, s, n, pos, vel, ids);
  if (s == 1) c->ncount_valid = false;
  if (s == 2) c->ion_moved_accum = 0;
  c->acc_next_valid = false;
  // The new population has no tile ranges yet: all of it bins as a tail.
  hipMemsetAsync(c->tsb[s][c->tcur[s]], 0, (c->ntiles + 1) * sizeof(uint32_t),
                 c->stream);
  c->n[s] = n;
  c->n_binned[s] = 0;
  k_set_n<<<1, 1, 0, c->stream>>>(c->dc, s, (unsigned long long)n);
  parts_bin_species(c, s);
  pic_status st = sync_counters(c);
  if (st != PIC_OK) return st;
  c->n[s] = (long long)c->hc.sorted_n[s];
  c->n_binned[s] = c->n[s];
  const long long hb[3] = {c->n[0], c->n[1], c->n[2]};
  parts_chunks(c, hb);
  if (c->hc.err) {
    check_flags(c);
    return set_err(c, PIC_ERR_ARG,
                   "particles outside the domain or non-finite were dropped");
  }
  return PIC_OK;
}

// ---- checkpoint ------------------------------------------------------------
namespace {

struct CkptHeader {
  char magic[8];
  int32_t abi, precision;
  int32_t nx, ny, nz, bc_lo, bc_hi, field_solve;
  double dx, v_lo, v_hi;
  uint64_t seed;
  uint32_t w_sp, pad;
  int64_t step;
  uint64_t next_id;
  int64_t n[PIC_NSPECIES];
  int32_t last_vcycles, hist_valid;  // bit 0: history, bit 1: u solved
  pic_collisions coll;
  pic_sources src;
  int64_t nnodes;
};
constexpr char kCkptMagic[8] = {'P', 'I', 'C', 'C', 'K', 'P', 'T', '2'};

size_t record_bytes(const pic_ctx* c) { return c->mixed ? 36 : 56; }

size_t ckpt_bytes(const pic_ctx* c) {
  size_t b = sizeof(CkptHeader);
  for (int s = 0; s < PIC_NSPECIES; ++s) b += (size_t)c->n[s] * record_bytes(c);
  // The potential and the one before it (extrapolated start).
  return b + 2 * (size_t)c->nnodes * sizeof(double);
}

}  // namespace

pic_status pic_checkpoint_bytes(pic_ctx* c, size_t* bytes) {
  if (!c || !bytes) return PIC_ERR_ARG;
  *bytes = ckpt_bytes(c);
  return PIC_OK;
}

pic_status pic_checkpoint_save(pic_ctx* c, void* host, size_t bytes) {
  if (!c || !host) return PIC_ERR_ARG;
  if (!c->queue.empty() || c->queue_used > 0)
    return set_err(c, PIC_ERR_STATE, "checkpoint with queued injections");
  if (bytes < ckpt_bytes(c))
    return set_err(c, PIC_ERR_ARG, "checkpoint buffer too small");
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kCkptMagic, 8);
  h.abi = PIC_ABI_VERSION;
  h.precision = c->cfg.precision;
  h.nx = c->cfg.nx; h.ny = c->cfg.ny; h.nz = c->cfg.nz;
  h.bc_lo = c->cfg.bc_lo; h.bc_hi = c->cfg.bc_hi;
  h.field_solve = c->cfg.field_solve;
  h.dx = c->cfg.dx; h.v_lo = c->cfg.v_lo; h.v_hi = c->cfg.v_hi;
  h.seed = c->cfg.seed;
  h.w_sp = c->cfg.w_sp;
  h.step = c->step;
  h.next_id = c->next_id;
  for (int s = 0; s < PIC_NSPECIES; ++s) h.n[s] = c->n[s];
  h.last_vcycles = c->last_vcycles;
  h.hist_valid = (c->hist_valid ? 1 : 0) | (c->u_solved ? 2 : 0);
  h.coll = c->coll;
  h.src = c->src;
  h.nnodes = c->nnodes;
  char* out = static_cast<char*>(host);
  std::memcpy(out, &h, sizeof(h));
  size_t off = sizeof(h);
  for (int s = 0; s < PIC_NSPECIES; ++s) {
    void* ptr[8];
    size_t elem[8];
    const int na = parts_arrays(c, s, ptr, elem);
    for (int k = 0; k < na; ++k) {
      const size_t nb = (size_t)c->n[s] * elem[k];
      if (nb && !hip_ok(c, hipMemcpyAsync(out + off, ptr[k], nb,
                                          hipMemcpyDeviceToHost, c->stream),
                        "checkpoint copy"))
        return PIC_ERR_HIP;
      off += nb;
    }
  }
  const size_t nb = (size_t)c->nnodes * sizeof(double);
  if (!hip_ok(c, hipMemcpyAsync(out + off, c->lev[0].u, nb,
                                hipMemcpyDeviceToHost, c->stream),
              "checkpoint copy") ||
      !hip_ok(c, hipMemcpyAsync(out + off + nb, c->phi_hist, nb,
                                hipMemcpyDeviceToHost, c->stream),
              "checkpoint copy") ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "synchronise"))
    return PIC_ERR_HIP;
  return PIC_OK;
}

pic_status pic_checkpoint_load(pic_ctx* c, const void* host, size_t bytes) {
  if (!c || !host || bytes < sizeof(CkptHeader)) return PIC_ERR_ARG;
  CkptHeader h;
  std::memcpy(&h, host, sizeof(h));
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.abi != PIC_ABI_VERSION)
    return set_err(c, PIC_ERR_ARG, "not a checkpoint of this library version");
  const pic_config& f = c->cfg;
  if (h.precision != f.precision || h.nx != f.nx || h.ny != f.ny ||
      h.nz != f.nz || h.bc_lo != f.bc_lo || h.bc_hi != f.bc_hi ||
      h.field_solve != f.field_solve || h.dx != f.dx || h.v_lo != f.v_lo ||
      h.v_hi != f.v_hi || h.seed != f.seed || h.w_sp != f.w_sp ||
      h.nnodes != c->nnodes)
    return set_err(c, PIC_ERR_ARG, "checkpoint of another configuration");
  for (int s = 0; s < PIC_NSPECIES; ++s)
    if (h.n[s] < 0 || h.n[s] > f.capacity[s])
      return set_err(c, PIC_ERR_CAPACITY, "checkpoint exceeds capacity");
  size_t need = sizeof(CkptHeader) + 2 * (size_t)c->nnodes * sizeof(double);
  for (int s = 0; s < PIC_NSPECIES; ++s) need += (size_t)h.n[s] * record_bytes(c);
  if (bytes < need) return set_err(c, PIC_ERR_ARG, "checkpoint truncated");
  pic_status st = pic_set_collisions(c, &h.coll);
  if (st == PIC_OK) st = pic_set_sources(c, &h.src);
  if (st != PIC_OK) return st;
  c->ncount_valid = false;  // the neutrals are replaced
  c->ion_moved_accum = 0;
  c->acc_next_valid = false;
  for (int s = 0; s < PIC_NSPECIES; ++s) c->n[s] = h.n[s];
  const char* in = static_cast<const char*>(host);
  size_t off = sizeof(h);
  for (int s = 0; s < PIC_NSPECIES; ++s) {
    void* ptr[8];
    size_t elem[8];
    const int na = parts_arrays(c, s, ptr, elem);
    for (int k = 0; k < na; ++k) {
      const size_t nb = (size_t)h.n[s] * elem[k];
      if (nb && !hip_ok(c, hipMemcpyAsync(ptr[k], in + off, nb,
                                          hipMemcpyHostToDevice, c->stream),
                        "restore copy"))
        return PIC_ERR_HIP;
      off += nb;
    }
  }
  const size_t nb = (size_t)c->nnodes * sizeof(double);
  if (!hip_ok(c, hipMemcpyAsync(c->lev[0].u, in + off, nb,
                                hipMemcpyHostToDevice, c->stream),
              "restore copy") ||
      !hip_ok(c, hipMemcpyAsync(c->phi_hist, in + off + nb, nb,
                                hipMemcpyHostToDevice, c->stream),
              "restore copy"))
    return PIC_ERR_HIP;
  c->hist_valid = (h.hist_valid & 1) != 0;
  c->u_solved = (h.hist_valid & 2) != 0;
  // Keys from the restored layout, then the binning pass as for a load.
  for (int s = 0; s < PIC_NSPECIES; ++s) {
    parts_restore_keys(c, s, h.n[s]);
    hipMemsetAsync(c->tsb[s][c->tcur[s]], 0, (c->ntiles + 1) * sizeof(uint32_t),
                   c->stream);
    c->n_binned[s] = 0;
    k_set_n<<<1, 1, 0, c->stream>>>(c->dc, s, (unsigned long long)h.n[s]);
    parts_bin_species(c, s);
  }
  st = sync_counters(c);
  if (st != PIC_OK) return st;
  for (int s = 0; s < PIC_NSPECIES; ++s) {
    c->n[s] = (long long)c->hc.sorted_n[s];
    c->n_binned[s] = c->n[s];
  }
  const long long hb[3] = {c->n[0], c->n[1], c->n[2]};
  parts_chunks(c, hb);
  c->step = h.step;
  c->next_id = h.next_id;
  c->last_vcycles = h.last_vcycles;
  c->queue.clear();
  c->queue_used = 0;
  if (c->hc.err) {
    check_flags(c);
    return set_err(c, PIC_ERR_ARG, "checkpoint holds particles outside the domain");
  }
  return hip_ok(c, hipStreamSynchronize(c->stream), "synchronise") ? PIC_OK : PIC_ERR_HIP;
}

pic_status pic_md_return(pic_ctx* c, double lattice_a, uint32_t mask,
                         int64_t cap, double* pos, double* vel, uint64_t* ids,
                         int32_t* species, int64_t* n) {
  if (!c || !n || !(lattice_a >= 0.0) || (mask & ~15u)) return PIC_ERR_ARG;
  if (c->step == 0) return set_err(c, PIC_ERR_STATE, "no step taken yet");
  long long tot = 0;
  for (int s = 0; s < PIC_NSPECIES; ++s)
    if ((mask >> s) & 1u) tot += (long long)c->hc.cathode[s];
  *n = tot;
  if (cap < tot) return set_err(c, PIC_ERR_CAPACITY, "output buffers too small");
  if (tot == 0) return PIC_OK;
  if (!pos || !vel || !ids) return PIC_ERR_ARG;
  parts_md_return(c, lattice_a, mask, pos, vel, ids, species, cap);
  if (!hip_ok(c, hipGetLastError(), "md return launch") ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "synchronise"))
    return PIC_ERR_HIP;
  return PIC_OK;
}

pic_status pic_debye_check(pic_ctx* c, int32_t block, double alpha_D,
                           double* lambda, pic_debye_info* info) {
  if (!c || !info) return PIC_ERR_ARG;
  if ((block != 1 && block != 2 && block != 4 && block != 8) ||
      c->cfg.nx % block || c->cfg.ny % block || c->cfg.nz % block ||
      !(alpha_D > 0.0) || !std::isfinite(alpha_D))
    return set_err(c, PIC_ERR_ARG, "block must be 1, 2, 4 or 8 and divide the grid");
  tmark(c, PIC_PH_DEBYE, true);
  parts_debye(c, block, alpha_D, lambda, c->dbg_out);
  tmark(c, PIC_PH_DEBYE, false);
  double out[4];
  if (!hip_ok(c, hipGetLastError(), "debye launch") ||
      !hip_ok(c, hipMemcpyAsync(out, c->dbg_out, sizeof(out),
                                hipMemcpyDeviceToHost, c->stream),
              "debye readback") ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "synchronise"))
    return PIC_ERR_HIP;
  collect_times(c);
  info->blocks = (int64_t)(c->cfg.nx / block) * (c->cfg.ny / block) *
                 (c->cfg.nz / block);
  info->checked = (int64_t)out[0];
  info->unresolved = (int64_t)out[1];
  info->lambda_min = out[2];
  info->ratio_max = out[3];
  return PIC_OK;
}

double pic_alpha_eh(double R, double d, double ell, double phi_w_eV,
                    double E_e_eV) {
  return ((1.0 - R) * (1.0 - std::exp(-d / ell))) * (1.0 - phi_w_eV / E_e_eV);
}

pic_status pic_count(pic_ctx* c, int32_t s, int64_t* n) {
  if (!c || s < 0 || s >= PIC_NSPECIES || !n) return PIC_ERR_ARG;
  *n = c->n[s];
  return PIC_OK;
}

pic_status pic_read_particles(pic_ctx* c, int32_t s, int64_t cap, double* pos,
                              double* vel, uint64_t* ids, int64_t* n) {
  if (!c || s < 0 || s >= PIC_NSPECIES) return PIC_ERR_ARG;
  if (n) *n = c->n[s];
  if (cap < c->n[s]) return set_err(c, PIC_ERR_CAPACITY, "read buffer small");
  if (c->n[s] > 0 && (!pos || !vel || !ids)) return PIC_ERR_ARG;
  parts_read(c, s, c->n[s], pos, vel, ids);
  if (!hip_ok(c, hipStreamSynchronize(c->stream), "read synchronise"))
    return PIC_ERR_HIP;
  return PIC_OK;
}

pic_status pic_read_fields(pic_ctx* c, int64_t* acc, double* phi, double* E3) {
  if (!c) return PIC_ERR_ARG;
  if (acc &&
      !hip_ok(c, hipMemcpyAsync(acc, c->acc, c->nnodes * sizeof(long long),
                                hipMemcpyDeviceToDevice, c->stream),
              "acc copy"))
    return PIC_ERR_HIP;
  if (phi &&
      !hip_ok(c, hipMemcpyAsync(phi, c->lev[0].u, c->nnodes * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream),
              "phi copy"))
    return PIC_ERR_HIP;
  if (E3) {
    const long long n = c->nnodes;
    k_deinterleave_E<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(
        reinterpret_cast<const char*>(c->E), c->mixed ? 1 : 0, E3, n);
  }
  if (!hip_ok(c, hipStreamSynchronize(c->stream), "read synchronise"))
    return PIC_ERR_HIP;
  return PIC_OK;
}

pic_status pic_set_clock(pic_ctx* c, int64_t step, uint64_t next_id) {
  if (!c || step < 0) return PIC_ERR_ARG;
  c->step = step;
  c->next_id = next_id;
  return PIC_OK;
}

pic_status pic_get_diag(pic_ctx* c, pic_diag* d) {
  if (!c || !d) return PIC_ERR_ARG;
  fill_diag(c, d);
  return PIC_OK;
}

}  // extern "C"
