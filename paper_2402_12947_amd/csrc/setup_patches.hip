// Local-correction subdomains (paper Sec. 4.1, Sec. 4.4 eq. identify).
//
// Omega_b = cells with gamma < tau (flags computed on the GPU).  The integer
// graph work over the flagged region runs on the host: components of Omega_b
// under "shares a vertex" (each started from its lowest cell id), growth by
// `layers` vertex layers, and under the MERGE policy the union of grown sets
// that share a vertex, so that subdomains have pairwise disjoint closures.
// Patches are ordered by their smallest cell id.  B_d = the free DOFs of the
// patch's cells (gathered from the device DOF map), ascending.  Colours: greedy
// in patch order over the "shares a DOF" conflict graph (MERGE gives one).
#include <algorithm>
#include <numeric>
#include <unordered_map>

#include "devutil.h"

namespace mg {

__global__ void k_gather_cell_free_dofs(const int32_t *cells, int64_t n, const int32_t *cell_dofs, int nloc,
                                        const int32_t *free_index, int32_t *out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nloc) return;
  int64_t k = t / nloc;
  int j = (int)(t - k * nloc);
  out[t] = free_index[cell_dofs[(int64_t)cells[k] * nloc + j]];
}

void build_patches(Ctx &c, Level &L, const mg_mesh &m) {
  hipStream_t s = c.stream;
  Patches &P = L.patch;
  std::vector<uint8_t> flags;
  download(flags, L.flags.p, (size_t)L.nc, s);
  std::vector<int32_t> flagged;
  for (int64_t i = 0; i < L.nc; ++i)
    if (flags[i]) flagged.push_back((int32_t)i);
  L.nflagged = (int64_t)flagged.size();
  P.n = 0;
  P.ncolour = 0;
  P.maxn = 0;
  P.total = 0;
  P.colour_first.assign(1, 0);
  P.h_ptr.assign(1, 0);
  P.h_dofs.clear();
  P.h_colour.clear();
  if (flagged.empty() || !c.opt.local_correction) return;

  const int nvert = L.dim + 1;
  const int32_t *cells = m.cells;
  // vertex -> cells
  std::vector<int64_t> vptr(L.nv + 1, 0);
  for (int64_t i = 0; i < L.nc * nvert; ++i) vptr[cells[i] + 1]++;
  for (int64_t v = 0; v < L.nv; ++v) vptr[v + 1] += vptr[v];
  std::vector<int32_t> vcell(vptr[L.nv]);
  {
    std::vector<int64_t> cur(vptr.begin(), vptr.end() - 1);
    for (int64_t cc = 0; cc < L.nc; ++cc)
      for (int a = 0; a < nvert; ++a) vcell[cur[cells[cc * nvert + a]]++] = (int32_t)cc;
  }
  // components of Omega_b
  std::vector<int32_t> stamp(L.nc, -1);
  std::vector<std::vector<int32_t>> comps;
  for (int32_t c0 : flagged) {
    if (stamp[c0] >= 0) continue;
    int id = (int)comps.size();
    std::vector<int32_t> comp, queue{c0};
    stamp[c0] = id;
    for (size_t qi = 0; qi < queue.size(); ++qi) {
      int32_t cc = queue[qi];
      comp.push_back(cc);
      for (int a = 0; a < nvert; ++a) {
        int32_t v = cells[(int64_t)cc * nvert + a];
        for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k) {
          int32_t nb = vcell[k];
          if (flags[nb] && stamp[nb] < 0) {
            stamp[nb] = id;
            queue.push_back(nb);
          }
        }
      }
    }
    std::sort(comp.begin(), comp.end());
    comps.push_back(std::move(comp));
  }
  // vertex-layer growth
  std::vector<int32_t> mark(L.nc, -1), vmark(L.nv, -1);
  std::vector<std::vector<int32_t>> grown(comps.size());
  int epoch = 0;
  for (size_t p = 0; p < comps.size(); ++p) {
    std::vector<int32_t> cur = comps[p];
    ++epoch;
    for (int32_t cc : cur) mark[cc] = epoch;
    for (int layer = 0; layer < c.layers; ++layer) {
      std::vector<int32_t> add;
      for (int32_t cc : cur)
        for (int a = 0; a < nvert; ++a) {
          int32_t v = cells[(int64_t)cc * nvert + a];
          if (vmark[v] == epoch) continue;
          vmark[v] = epoch;
          for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k)
            if (mark[vcell[k]] != epoch) {
              mark[vcell[k]] = epoch;
              add.push_back(vcell[k]);
            }
        }
      cur.insert(cur.end(), add.begin(), add.end());
    }
    std::sort(cur.begin(), cur.end());
    grown[p] = std::move(cur);
  }
  // merge grown sets sharing a vertex (union-find)
  std::vector<std::vector<int32_t>> sets;
  if (c.opt.patch_policy == MG_PATCH_MERGE) {
    std::vector<int> parent(grown.size());
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int a) {
      while (parent[a] != a) {
        parent[a] = parent[parent[a]];
        a = parent[a];
      }
      return a;
    };
    std::vector<int32_t> owner(L.nv, -1);
    for (size_t p = 0; p < grown.size(); ++p)
      for (int32_t cc : grown[p])
        for (int a = 0; a < nvert; ++a) {
          int32_t v = cells[(int64_t)cc * nvert + a];
          if (owner[v] < 0) {
            owner[v] = (int32_t)p;
          } else {
            int ra = find(owner[v]), rb = find((int)p);
            if (ra != rb) parent[std::max(ra, rb)] = std::min(ra, rb);
          }
        }
    std::unordered_map<int, size_t> slot;
    for (size_t p = 0; p < grown.size(); ++p) {
      int r = find((int)p);
      auto it = slot.find(r);
      if (it == slot.end()) {
        slot[r] = sets.size();
        sets.push_back(grown[p]);
      } else {
        auto &dst = sets[it->second];
        dst.insert(dst.end(), grown[p].begin(), grown[p].end());
      }
    }
    for (auto &st : sets) {
      std::sort(st.begin(), st.end());
      st.erase(std::unique(st.begin(), st.end()), st.end());
    }
  } else {
    sets = grown;
  }
  std::stable_sort(sets.begin(), sets.end(),
                   [](const std::vector<int32_t> &a, const std::vector<int32_t> &b) { return a[0] < b[0]; });
  // DOF sets from the device DOF map
  std::vector<int32_t> allcells;
  for (auto &st : sets) allcells.insert(allcells.end(), st.begin(), st.end());
  DBuf<int32_t> dcells, dout;
  upload(dcells, allcells.data(), allcells.size(), s);
  dout.alloc(allcells.size() * L.nloc);
  k_gather_cell_free_dofs<<<grid_for((int64_t)allcells.size() * L.nloc, 256), 256, 0, s>>>(
      dcells, (int64_t)allcells.size(), L.cell_dofs, L.nloc, L.free_index, dout);
  MG_LAUNCH_CHECK();
  std::vector<int32_t> fd;
  download(fd, dout.p, allcells.size() * L.nloc, s);
  std::vector<std::vector<int32_t>> dofs;
  size_t pos = 0;
  for (auto &st : sets) {
    std::vector<int32_t> d;
    for (size_t k = 0; k < st.size() * L.nloc; ++k)
      if (fd[pos + k] >= 0) d.push_back(fd[pos + k]);
    pos += st.size() * L.nloc;
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
    if (L.ncomp > 1) {  // every component of the patch's DOF nodes: s * ncomp + c
      std::vector<int32_t> v;
      v.reserve(d.size() * L.ncomp);
      for (int32_t x : d)
        for (int k = 0; k < L.ncomp; ++k) v.push_back(x * L.ncomp + k);
      d.swap(v);
    }
    if (!d.empty()) dofs.push_back(std::move(d));
  }
  set_patches(c, L, dofs);
}

// The level's patches from their DOF sets (canonical free ids, ascending, in
// patch order): greedy colours, export arrays, kernel order, packed layout.
void set_patches(Ctx &c, Level &L, const std::vector<std::vector<int32_t>> &dofs) {
  hipStream_t s = c.stream;
  Patches &P = L.patch;
  P.h_ptr.assign(1, 0);
  P.h_dofs.clear();
  P.h_colour.clear();
  P.maxn = 0;
  // greedy colouring over shared DOFs
  std::unordered_map<int32_t, std::vector<int>> owners;
  std::vector<int> colour(dofs.size(), 0);
  int ncol = 0;
  for (size_t p = 0; p < dofs.size(); ++p) {
    std::vector<char> used;
    for (int32_t d : dofs[p]) {
      auto it = owners.find(d);
      if (it == owners.end()) continue;
      for (int q : it->second) {
        if ((size_t)colour[q] >= used.size()) used.resize(colour[q] + 1, 0);
        used[colour[q]] = 1;
      }
    }
    int col = 0;
    while ((size_t)col < used.size() && used[col]) ++col;
    colour[p] = col;
    ncol = std::max(ncol, col + 1);
    for (int32_t d : dofs[p]) owners[d].push_back((int)p);
  }
  // canonical-order export arrays
  P.n = (int)dofs.size();
  P.ncolour = ncol;
  P.h_ptr.assign(P.n + 1, 0);
  for (int p = 0; p < P.n; ++p) {
    P.h_ptr[p + 1] = P.h_ptr[p] + (int32_t)dofs[p].size();
    P.h_dofs.insert(P.h_dofs.end(), dofs[p].begin(), dofs[p].end());
    P.h_colour.push_back(colour[p]);
    P.maxn = std::max(P.maxn, (int)dofs[p].size());
  }
  P.total = P.h_ptr[P.n];
  if (P.maxn > MAX_PATCH)
    fail(MG_ERR_LIMIT, "a local-correction patch has %d DOFs (limit %d): the low-quality regions merge into "
                       "one large subdomain%s", P.maxn, MAX_PATCH,
         P.n_inherited > 0 ? " (with the patches inherited from the finer level; fewer patch_inherit_levels "
                             "avoid it)" : "");
  // kernel order: by colour, then canonical id
  std::vector<int> order(P.n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return colour[a] < colour[b]; });
  std::vector<int32_t> kptr(P.n + 1, 0), kdofs;
  std::vector<int64_t> off(P.n, 0);
  P.colour_first.assign(ncol + 1, P.n);
  int64_t acc = 0;
  for (int k = 0; k < P.n; ++k) {
    int p = order[k];
    if (k == 0 || colour[order[k - 1]] != colour[p]) P.colour_first[colour[p]] = k;
    kptr[k + 1] = kptr[k] + (int32_t)dofs[p].size();
    kdofs.insert(kdofs.end(), dofs[p].begin(), dofs[p].end());
    off[k] = acc;
    acc += (int64_t)dofs[p].size() * (int64_t)dofs[p].size();
  }
  P.colour_first[ncol] = P.n;
  build_packed_layout(s, kptr, P.colour_first, P.inv);
  P.h_kptr = kptr;
  upload(P.ptr, kptr.data(), kptr.size(), s);
  upload(P.dofs_canon, kdofs.data(), kdofs.size(), s);
  upload(P.inv_off, off.data(), off.size(), s);
  P.inv64.alloc(acc);
  MG_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// patches inherited through the transfer operators
// ---------------------------------------------------------------------------
// seeds: the free DOFs of each degraded cell of level 0 (every component for
// vector problems), one set per cell in cell order
void patch_seeds(Ctx &c, Level &L, std::vector<std::vector<int32_t>> &seeds) {
  hipStream_t s = c.stream;
  std::vector<uint8_t> flags;
  download(flags, L.flags.p, (size_t)L.nc, s);
  std::vector<int32_t> flagged;
  for (int64_t i = 0; i < L.nc; ++i)
    if (flags[i]) flagged.push_back((int32_t)i);
  seeds.clear();
  if (flagged.empty()) return;
  DBuf<int32_t> dcells, dout;
  upload(dcells, flagged.data(), flagged.size(), s);
  dout.alloc(flagged.size() * L.nloc);
  k_gather_cell_free_dofs<<<grid_for((int64_t)flagged.size() * L.nloc, 256), 256, 0, s>>>(
      dcells, (int64_t)flagged.size(), L.cell_dofs, L.nloc, L.free_index, dout);
  MG_LAUNCH_CHECK();
  std::vector<int32_t> fd;
  download(fd, dout.p, flagged.size() * L.nloc, s);
  for (size_t k = 0; k < flagged.size(); ++k) {
    std::vector<int32_t> d;
    for (int j = 0; j < L.nloc; ++j)
      if (fd[k * L.nloc + j] >= 0) d.push_back(fd[k * L.nloc + j]);
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
    if (L.ncomp > 1) {
      std::vector<int32_t> v;
      for (int32_t x : d)
        for (int q = 0; q < L.ncomp; ++q) v.push_back(x * L.ncomp + q);
      d.swap(v);
    }
    seeds.push_back(std::move(d));
  }
}

__global__ void k_gather_rows(const int32_t *pcol, int width, const int32_t *rows, int64_t n, int32_t *out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * width) return;
  out[t] = pcol[(int64_t)rows[t / width] * width + t % width];
}

// union-find over a family of DOF sets joined by shared DOFs; root = the
// lowest index of the group
static std::vector<int> join_sharing(const std::vector<std::vector<int32_t>> &sets) {
  std::vector<int> parent(sets.size());
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int a) {
    while (parent[a] != a) {
      parent[a] = parent[parent[a]];
      a = parent[a];
    }
    return a;
  };
  std::unordered_map<int32_t, int> owner;
  for (size_t k = 0; k < sets.size(); ++k)
    for (int32_t d : sets[k]) {
      auto it = owner.find(d);
      if (it == owner.end()) {
        owner.emplace(d, (int)k);
      } else {
        int ra = find(it->second), rb = find((int)k);
        if (ra != rb) parent[std::max(ra, rb)] = std::min(ra, rb);
      }
    }
  for (size_t k = 0; k < sets.size(); ++k) parent[k] = find((int)k);
  return parent;
}

// seeds of fine level F -> the coarse DOFs its interpolation couples to them
// (per set: the columns of P's rows at the set, i.e. the free DOFs of the
// coarse cells containing the nodes); the connected components of those sets
// join coarse level C's own patches (MERGE: components sharing DOFs with own
// patches merge into the lowest-indexed one; OVERLAP: appended and coloured).
void inherit_patches(Ctx &c, const Level &F, Level &C, std::vector<std::vector<int32_t>> &seeds) {
  hipStream_t s = c.stream;
  std::vector<int32_t> rows;
  for (auto &st : seeds) rows.insert(rows.end(), st.begin(), st.end());
  std::vector<int32_t> pc;
  if (!rows.empty()) {
    DBuf<int32_t> drows, dout;
    upload(drows, rows.data(), rows.size(), s);
    dout.alloc(rows.size() * F.pw);
    k_gather_rows<<<grid_for((int64_t)rows.size() * F.pw, 256), 256, 0, s>>>(F.pcol, F.pw, drows,
                                                                             (int64_t)rows.size(), dout);
    MG_LAUNCH_CHECK();
    download(pc, dout.p, rows.size() * F.pw, s);
  }
  std::vector<std::vector<int32_t>> next;
  size_t pos = 0;
  for (auto &st : seeds) {
    std::vector<int32_t> d;
    for (size_t k = 0; k < st.size() * F.pw; ++k)
      if (pc[pos * F.pw + k] >= 0) d.push_back(pc[pos * F.pw + k]);
    pos += st.size();
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
    next.push_back(std::move(d));
  }
  seeds.swap(next);
  // components of the inherited sets, ordered by smallest DOF
  std::vector<int> root = join_sharing(seeds);
  std::vector<std::vector<int32_t>> comps;
  std::unordered_map<int, size_t> slot;
  for (size_t k = 0; k < seeds.size(); ++k) {
    if (seeds[k].empty()) continue;
    auto it = slot.find(root[k]);
    if (it == slot.end()) {
      slot.emplace(root[k], comps.size());
      comps.push_back(seeds[k]);
    } else {
      auto &dst = comps[it->second];
      dst.insert(dst.end(), seeds[k].begin(), seeds[k].end());
    }
  }
  for (auto &cp : comps) {
    std::sort(cp.begin(), cp.end());
    cp.erase(std::unique(cp.begin(), cp.end()), cp.end());
  }
  std::sort(comps.begin(), comps.end(),
            [](const std::vector<int32_t> &a, const std::vector<int32_t> &b) { return a[0] < b[0]; });
  // own patches, then the components
  const Patches &P = C.patch;
  std::vector<std::vector<int32_t>> all;
  for (int p = 0; p < P.n; ++p) all.emplace_back(P.h_dofs.begin() + P.h_ptr[p], P.h_dofs.begin() + P.h_ptr[p + 1]);
  const size_t nown = all.size();
  for (auto &cp : comps) all.push_back(cp);
  std::vector<std::vector<int32_t>> out;
  if (c.opt.patch_policy == MG_PATCH_MERGE) {
    std::vector<int> r = join_sharing(all);
    std::unordered_map<int, size_t> at;
    for (size_t k = 0; k < all.size(); ++k) {
      auto it = at.find(r[k]);
      if (it == at.end()) {
        at.emplace(r[k], out.size());
        out.push_back(all[k]);
      } else {
        auto &dst = out[it->second];
        dst.insert(dst.end(), all[k].begin(), all[k].end());
      }
    }
    for (auto &o : out) {
      std::sort(o.begin(), o.end());
      o.erase(std::unique(o.begin(), o.end()), o.end());
    }
  } else {
    out = std::move(all);
  }
  C.patch.n_inherited = (int)comps.size();
  (void)nown;
  set_patches(c, C, out);
}


__global__ void k_map_dofs(const int32_t *canon, int64_t n, const int32_t *iperm, int32_t *pos) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) pos[k] = iperm[canon[k]];
}

// Item lists and offsets of a set of packed symmetric inverses; kptr[k]..kptr[k+1]
// is the index range of system k, colour_first the system ranges per colour.
void build_packed_layout(hipStream_t s, const std::vector<int32_t> &kptr, const std::vector<int> &colour_first,
                         PackedInv &P, int chunk) {
  P.chunk = chunk;
  const int ns = (int)kptr.size() - 1, ncol = (int)colour_first.size() - 1;
  std::vector<int64_t> toff(ns), zoff(ns);
  std::vector<int32_t> rs, rr, rc, rslot, gs, gr, gslot;
  int64_t tacc = 0, zacc = 0;
  int32_t slot = 0;
  P.colour_r_first.assign(ncol + 1, 0);
  P.colour_g_first.assign(ncol + 1, 0);
  for (int col = 0; col < ncol; ++col) {
    P.colour_r_first[col] = (int)rs.size();
    P.colour_g_first[col] = (int)gs.size();
    for (int k = colour_first[col]; k < colour_first[col + 1]; ++k) {
      int64_t nb = (kptr[k + 1] - kptr[k] + PATCH_TILE - 1) / PATCH_TILE;
      toff[k] = tacc;
      zoff[k] = zacc;
      tacc += nb * (nb + 1) / 2 * PATCH_TILE * PATCH_TILE;
      zacc += nb * (nb - 1) / 2 * PATCH_TILE;
      for (int64_t I = 0; I < nb; ++I) {
        gs.push_back(k);
        gr.push_back((int32_t)I);
        gslot.push_back(slot);
        for (int64_t c = 0; c * chunk <= I; ++c) {
          rs.push_back(k);
          rr.push_back((int32_t)I);
          rc.push_back((int32_t)c);
          rslot.push_back(slot++);
        }
      }
    }
  }
  P.colour_r_first[ncol] = (int)rs.size();
  P.colour_g_first[ncol] = (int)gs.size();
  // within a colour, row items with the most tiles first: they are launched
  // first, and the short items fill in behind them instead of leaving a tail
  // of long ones (each item writes only its own slot, so the order of the
  // items changes no result)
  for (int col = 0; col < ncol; ++col) {
    const int a = P.colour_r_first[col], b = P.colour_r_first[col + 1];
    std::vector<int> ord(b - a);
    for (int q = 0; q < b - a; ++q) ord[q] = a + q;
    auto tiles = [&](int q) { return std::min(rr[q] + 1, (rc[q] + 1) * chunk) - rc[q] * chunk; };
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return tiles(x) > tiles(y); });
    std::vector<int32_t> t0(b - a), t1(b - a), t2(b - a), t3(b - a);
    for (int q = 0; q < b - a; ++q) {
      t0[q] = rs[ord[q]];
      t1[q] = rr[ord[q]];
      t2[q] = rc[ord[q]];
      t3[q] = rslot[ord[q]];
    }
    std::copy(t0.begin(), t0.end(), rs.begin() + a);
    std::copy(t1.begin(), t1.end(), rr.begin() + a);
    std::copy(t2.begin(), t2.end(), rc.begin() + a);
    std::copy(t3.begin(), t3.end(), rslot.begin() + a);
  }
  P.packed = tacc;
  P.ysize = (int64_t)slot * PATCH_TILE;
  P.zsize = zacc;
  upload(P.tile_off, toff.data(), toff.size(), s);
  upload(P.zoff, zoff.data(), zoff.size(), s);
  upload(P.r_sys, rs.data(), rs.size(), s);
  upload(P.r_row, rr.data(), rr.size(), s);
  upload(P.r_chunk, rc.data(), rc.size(), s);
  upload(P.r_slot, rslot.data(), rslot.size(), s);
  upload(P.g_sys, gs.data(), gs.size(), s);
  upload(P.g_row, gr.data(), gr.size(), s);
  upload(P.g_slot, gslot.data(), gslot.size(), s);
  MG_HIP(hipStreamSynchronize(s));
}

// patch DOFs in the level's solve order (after solve_order has set iperm)
void permute_patches(Ctx &c, Level &L) {
  Patches &P = L.patch;
  if (P.total == 0) return;
  P.dofs.alloc(P.total);
  k_map_dofs<<<grid_for(P.total, 256), 256, 0, c.stream>>>(P.dofs_canon, P.total, L.iperm, P.dofs);
  MG_LAUNCH_CHECK();
  MG_HIP(hipStreamSynchronize(c.stream));
}

}  // namespace mg
