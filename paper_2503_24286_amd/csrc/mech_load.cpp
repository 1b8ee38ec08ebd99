// Loader of .pyromech version-1 mechanism files and builder of the device
// tables the kernels read.
//
// File layout (little endian): a 48-byte header
//   char[8] "PYROMECH", u32 version (1), u32 S, u32 R, u32 E,
//   u32 n_third_body, u32 n_falloff, u32 reactant nnz, u32 product nnz,
//   u64 payload bytes,
// the payload arrays, each zero padded to 8 bytes,
//   f64 element_weight[E], i32 composition[E][S], f64 W[S],
//   f64 T_range[S][3] (T_low, T_mid, T_high), f64 nasa[S][2][7],
//   i32 rtype[R] (0 elementary, 1 third-body, 2 Lindemann, 3 Troe),
//   i32 reversible[R], f64 arrhenius[R][3] (ln A, b, Ea in J/mol),
//   i32 reac_ptr[R+1], reac_species[nnz], reac_nu[nnz],
//   i32 prod_ptr[R+1], prod_species[nnz], prod_nu[nnz],
//   i32 falloff_reaction[n_falloff], f64 falloff_low[n_falloff][3],
//   f64 troe[n_falloff][4] (alpha, T***, T*, T**),
//   f64 efficiency[n_third_body + n_falloff][S],
// and a trailing u64 FNV-1a hash of every preceding byte.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>

#include "pyro_internal.h"

namespace pyro {
namespace {

struct Reader {
    const uint8_t* data;
    size_t size;
    size_t pos;
    bool ok = true;

    template <class T>
    std::vector<T> take(size_t count) {
        std::vector<T> out(count);
        const size_t bytes = count * sizeof(T);
        if (!ok || pos + bytes > size) {
            ok = false;
            return out;
        }
        if (bytes) std::memcpy(out.data(), data + pos, bytes);
        pos += bytes + ((8 - bytes % 8) % 8);
        return out;
    }
};

uint64_t fnv1a64(const uint8_t* p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

bool all_finite(const std::vector<double>& v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

// Parsed file contents, in file order.
struct Parsed {
    uint32_t S, R, E, n_tb, n_fo;
    std::vector<double> ew, W, trange, nasa, arrh, low, troe, eff;
    std::vector<int32_t> comp, rtype, rev, rp, rs, rn, pp, ps, pn, fo;
};

int parse(const std::vector<uint8_t>& blob, Parsed& f) {
    if (blob.size() < 56) return fail(PYRO_E_FORMAT, "mechanism file too short");
    if (std::memcmp(blob.data(), "PYROMECH", 8) != 0)
        return fail(PYRO_E_FORMAT, "bad magic (not a .pyromech file)");
    uint32_t hdr[8];
    uint64_t payload;
    std::memcpy(hdr, blob.data() + 8, 32);
    std::memcpy(&payload, blob.data() + 40, 8);
    if (hdr[0] != 1)
        return fail(PYRO_E_FORMAT, "unsupported .pyromech version " + std::to_string(hdr[0]));
    if (payload > blob.size() || blob.size() != 48 + payload + 8)
        return fail(PYRO_E_FORMAT, "file size does not match the header");
    uint64_t stored;
    std::memcpy(&stored, blob.data() + 48 + payload, 8);
    if (stored != fnv1a64(blob.data(), 48 + payload))
        return fail(PYRO_E_FORMAT, "checksum mismatch (corrupted file)");
    f.S = hdr[1];
    f.R = hdr[2];
    f.E = hdr[3];
    f.n_tb = hdr[4];
    f.n_fo = hdr[5];
    const uint32_t nnz_r = hdr[6], nnz_p = hdr[7];
    if (f.S == 0 || f.S > 4096 || f.R > (1u << 20) || f.E > 64 ||
        f.n_tb + f.n_fo > f.R || nnz_r > 16 * (f.R + 1) || nnz_p > 16 * (f.R + 1))
        return fail(PYRO_E_FORMAT, "implausible counts in the header");
    Reader rd{blob.data(), 48 + payload, 48};
    f.ew = rd.take<double>(f.E);
    f.comp = rd.take<int32_t>(size_t(f.E) * f.S);
    f.W = rd.take<double>(f.S);
    f.trange = rd.take<double>(size_t(f.S) * 3);
    f.nasa = rd.take<double>(size_t(f.S) * 14);
    f.rtype = rd.take<int32_t>(f.R);
    f.rev = rd.take<int32_t>(f.R);
    f.arrh = rd.take<double>(size_t(f.R) * 3);
    f.rp = rd.take<int32_t>(f.R + 1);
    f.rs = rd.take<int32_t>(nnz_r);
    f.rn = rd.take<int32_t>(nnz_r);
    f.pp = rd.take<int32_t>(f.R + 1);
    f.ps = rd.take<int32_t>(nnz_p);
    f.pn = rd.take<int32_t>(nnz_p);
    f.fo = rd.take<int32_t>(f.n_fo);
    f.low = rd.take<double>(size_t(f.n_fo) * 3);
    f.troe = rd.take<double>(size_t(f.n_fo) * 4);
    f.eff = rd.take<double>(size_t(f.n_tb + f.n_fo) * f.S);
    if (!rd.ok || rd.pos != 48 + payload)
        return fail(PYRO_E_FORMAT, "payload size does not match the header counts");

    // values
    for (double w : f.W)
        if (!(std::isfinite(w) && w > 0)) return fail(PYRO_E_FORMAT, "non-positive or non-finite molar mass");
    if (!all_finite(f.ew) || !all_finite(f.trange) || !all_finite(f.nasa) ||
        !all_finite(f.arrh) || !all_finite(f.low) || !all_finite(f.troe) || !all_finite(f.eff))
        return fail(PYRO_E_FORMAT, "non-finite parameter in the mechanism");
    for (uint32_t k = 0; k < f.S; ++k) {
        const double* t = &f.trange[3 * k];
        if (!(t[0] > 0 && t[0] < t[1] && t[1] < t[2]))
            return fail(PYRO_E_FORMAT, "species " + std::to_string(k) + ": bad NASA7 temperature ranges");
    }
    uint32_t n_tb = 0, n_fo = 0;
    for (uint32_t j = 0; j < f.R; ++j) {
        if (f.rtype[j] < 0 || f.rtype[j] > 3)
            return fail(PYRO_E_FORMAT, "reaction " + std::to_string(j) + ": unknown class");
        if (f.rev[j] != 0 && f.rev[j] != 1)
            return fail(PYRO_E_FORMAT, "reaction " + std::to_string(j) + ": bad reversible flag");
        n_tb += f.rtype[j] == 1;
        n_fo += f.rtype[j] >= 2;
    }
    if (n_tb != f.n_tb || n_fo != f.n_fo)
        return fail(PYRO_E_FORMAT, "reaction classes do not match the header counts");
    auto check_csr = [&](const std::vector<int32_t>& ptr, const std::vector<int32_t>& sp,
                         const std::vector<int32_t>& nu, const char* side) -> int {
        if (ptr[0] != 0 || size_t(ptr[f.R]) != sp.size())
            return fail(PYRO_E_FORMAT, std::string(side) + " list pointers are inconsistent");
        for (uint32_t j = 0; j < f.R; ++j) {
            if (ptr[j + 1] < ptr[j])
                return fail(PYRO_E_FORMAT, std::string(side) + " list pointers decrease");
            for (int32_t q = ptr[j]; q < ptr[j + 1]; ++q) {
                if (sp[q] < 0 || uint32_t(sp[q]) >= f.S)
                    return fail(PYRO_E_FORMAT, std::string(side) + " species index out of range");
                if (nu[q] < 1 || nu[q] > 16)
                    return fail(PYRO_E_FORMAT, std::string(side) + " stoichiometric coefficient out of range");
            }
        }
        return PYRO_OK;
    };
    if (int rc = check_csr(f.rp, f.rs, f.rn, "reactant")) return rc;
    if (int rc = check_csr(f.pp, f.ps, f.pn, "product")) return rc;
    for (uint32_t i = 0, j = 0; j < f.R; ++j) {
        if (f.rtype[j] >= 2) {
            if (f.fo[i] != int32_t(j))
                return fail(PYRO_E_FORMAT, "falloff reaction list does not match the classes");
            ++i;
        }
    }
    for (uint32_t i = 0; i < f.n_fo; ++i) {
        const double* t = &f.troe[4 * i];
        if (f.rtype[f.fo[i]] == 3 && !(t[1] > 0 && t[2] > 0 && t[3] >= 0))
            return fail(PYRO_E_FORMAT, "Troe temperatures must be positive");
    }
    return PYRO_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct SchedInput {
    int S, R;
    const std::vector<int32_t>* rtype;
    const std::vector<int32_t>* rev;
    const std::vector<std::vector<int>>* reac;
    const std::vector<std::vector<int>>* prod;
    const std::vector<int>* dnu;
    const std::vector<int>* pd_row;
    const std::vector<int>* fo_idx;
    const std::vector<std::vector<std::pair<int, double>>>* by_species;
};

// A work schedule of one 64-cell tile over `waves` wavefronts: species
// ownership (who gathers which species' sums, at most own_cap per wave) and
// reactions dealt in chunks of waves * rpw slots, costliest first, each chunk
// balanced over the waves.
struct HostSched {
    int waves = 0, rpw = 0, n_chunks = 0, max_own = 0, max_pdw = 0;
    std::vector<RxnRec> recs;                    // [n_chunks][waves][rpw]
    std::vector<std::vector<int>> own, pd_of_wave;
    std::vector<int> slot_of, chunk_of;
};

// row_bytes: the kernel's LDS bytes per species row; participants' offsets
// in the reaction records are species * row_bytes
// rank_bias > 0 skews species ownership toward low wave indices: of the
// waves sharing a SIMD (w, w + 4, ...), the SIMD's arbiter issues the older
// ones first, so they reach each chunk barrier early and can take more of the
// gathering (weight 1 + rank_bias * (w / 4) on a wave's load)
int build_schedule(const SchedInput& in, int waves, int rpw, int own_cap, int row_bytes,
                   double rank_bias, const std::vector<std::vector<int>>& gathered,
                   HostSched& out) {
    const int S = in.S, R = in.R;
    const auto& rtype = *in.rtype;
    const auto& by_species = *in.by_species;
    out.waves = waves;
    out.rpw = rpw;
    // species ownership: balance the gathering work over the waves
    std::vector<int> order(S);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return by_species[a].size() > by_species[b].size();
    });
    out.own.assign(waves, {});
    std::vector<double> load(waves, 0.0);
    for (int k : order) {
        int best = -1;
        for (int w = 0; w < waves; ++w)
            if (int(out.own[w].size()) < own_cap &&
                (best < 0 || load[w] * (1.0 + rank_bias * (w / 4)) <
                                 load[best] * (1.0 + rank_bias * (best / 4))))
                best = w;
        if (best < 0) return fail(PYRO_E_UNSUPPORTED, "too many species for one workgroup");
        out.own[best].push_back(k);
        load[best] += 2.0 + double(by_species[k].size());
    }
    for (auto& o : out.own) std::sort(o.begin(), o.end());
    out.max_own = 0;
    for (auto& o : out.own) out.max_own = std::max<int>(out.max_own, int(o.size()));

    auto cost = [&](int j) {
        double c = 1.0 + ((*in.rev)[j] ? 0.5 : 0.0);
        if (rtype[j] >= 1) c += S / 24.0;
        if (rtype[j] == 2) c += 1.5;
        if (rtype[j] == 3) c += 6.0;
        return c;
    };
    std::vector<int> rorder(R);
    std::iota(rorder.begin(), rorder.end(), 0);
    std::stable_sort(rorder.begin(), rorder.end(), [&](int a, int b) { return cost(a) > cost(b); });
    const int chunk = waves * rpw;
    out.n_chunks = (R + chunk - 1) / chunk;
    // chunk membership: by cost rank, then pairwise swaps of reactions of the
    // same cost class between chunks while they lower the sum over chunks of
    // the largest per-wave gathering load (each chunk ends at a barrier)
    std::vector<int> chunk_of(R);
    for (int t = 0; t < R; ++t) chunk_of[rorder[t]] = t / chunk;
    std::vector<int> owner(S, 0);
    for (int w = 0; w < waves; ++w)
        for (int k : out.own[w]) owner[k] = w;
    std::vector<std::vector<int>> contrib(R, std::vector<int>(waves, 0));
    for (int j = 0; j < R; ++j)
        for (int k : gathered[j]) contrib[j][owner[k]]++;
    std::vector<std::vector<int>> load_cw(std::max(out.n_chunks, 1), std::vector<int>(waves, 0));
    for (int j = 0; j < R; ++j)
        for (int w = 0; w < waves; ++w) load_cw[chunk_of[j]][w] += contrib[j][w];
    auto max_after = [&](int c, int rm, int add) {
        int mx = 0;
        for (int w = 0; w < waves; ++w)
            mx = std::max(mx, load_cw[c][w] - contrib[rm][w] + contrib[add][w]);
        return mx;
    };
    auto cmax = [&](int c) { return *std::max_element(load_cw[c].begin(), load_cw[c].end()); };
    auto same_class = [&](int a, int b) { return rtype[a] == rtype[b] && (*in.rev)[a] == (*in.rev)[b]; };
    for (int sweep = 0; sweep < 8; ++sweep) {
        bool improved = false;
        for (int a = 0; a < R; ++a)
            for (int b = a + 1; b < R; ++b) {
                const int ca = chunk_of[a], cb = chunk_of[b];
                if (ca == cb || !same_class(a, b)) continue;
                const int delta = max_after(ca, a, b) + max_after(cb, b, a) - cmax(ca) - cmax(cb);
                if (delta >= 0) continue;
                for (int w = 0; w < waves; ++w) {
                    load_cw[ca][w] += contrib[b][w] - contrib[a][w];
                    load_cw[cb][w] += contrib[a][w] - contrib[b][w];
                }
                std::swap(chunk_of[a], chunk_of[b]);
                improved = true;
            }
        if (!improved) break;
    }
    std::vector<std::vector<int>> members(std::max(out.n_chunks, 1));
    for (int t = 0; t < R; ++t) members[chunk_of[rorder[t]]].push_back(rorder[t]);
    out.recs.assign(size_t(std::max(out.n_chunks, 1)) * chunk, RxnRec{});
    for (auto& r : out.recs) {
        std::memset(&r, 0, sizeof(r));
        r.cls = kNoReaction;
    }
    out.slot_of.assign(R, -1);
    out.chunk_of.assign(R, -1);
    out.pd_of_wave.assign(waves, {});
    for (int c = 0; c < out.n_chunks; ++c) {
        std::vector<double> wl(waves, 0.0);
        std::vector<int> used(waves, 0);
        for (int j : members[c]) {
            const bool is_pd = rtype[j] >= 1;
            int best = -1;
            for (int w = 0; w < waves; ++w)
                if (used[w] < rpw && !(is_pd && int(out.pd_of_wave[w].size()) == kMaxPd) &&
                    (best < 0 || wl[w] < wl[best]))
                    best = w;
            if (best < 0) return fail(PYRO_E_UNSUPPORTED, "too many third-body and falloff reactions");
            const int slot = best * rpw + used[best]++;
            if (is_pd) out.pd_of_wave[best].push_back(j);
            wl[best] += cost(j);
            out.slot_of[j] = slot;
            out.chunk_of[j] = c;
            RxnRec& r = out.recs[size_t(c) * chunk + slot];
            const auto& rj = (*in.reac)[j];
            const auto& pj = (*in.prod)[j];
            r.cls = rtype[j];
            r.rev = (*in.rev)[j];
            r.nr = int(rj.size());
            r.np = int(pj.size());
            for (int s = 0; s < kMaxSide; ++s) {
                r.r[s] = s < r.nr ? rj[s] * row_bytes : 0;
                r.p[s] = s < r.np ? pj[s] * row_bytes : 0;
            }
            r.dnu = (*in.dnu)[j];
            r.prow = j;
            r.pdw = is_pd ? int(out.pd_of_wave[best].size()) - 1 : -1;
            r.fo = (*in.fo_idx)[j];
            r.qoff = slot * kTile * 8;
            r.pd = (*in.pd_row)[j];
        }
    }
    out.max_pdw = 0;
    for (auto& p : out.pd_of_wave) out.max_pdw = std::max<int>(out.max_pdw, int(p.size()));
    return PYRO_OK;
}

// The schedule of one Jacobian row (the reverse sweep with the cotangent on
// one species): only the reactions in ``subset`` (those whose net
// coefficient of that species is nonzero; every other reaction has a zero
// cotangent), costliest first, packed into as few chunks of ``waves`` slots
// as they fill (one reaction per wave per chunk), each chunk balanced over
// the waves.  Species ownership is the given one (that of the full reverse
// sweep, whose per-wave tables the row shares); a wave takes at most
// ``pd_cap`` third-body and falloff reactions.
int build_row_schedule(const SchedInput& in, const std::vector<int>& subset,
                       const std::vector<std::vector<int>>& own, int waves, int row_bytes,
                       int pd_cap, HostSched& out) {
    const int S = in.S, R = in.R;
    const auto& rtype = *in.rtype;
    out.waves = waves;
    out.rpw = 1;
    out.own = own;
    out.max_own = 0;
    for (auto& o : out.own) out.max_own = std::max<int>(out.max_own, int(o.size()));
    auto cost = [&](int j) {
        double c = 1.0 + ((*in.rev)[j] ? 0.5 : 0.0);
        if (rtype[j] >= 1) c += S / 24.0;
        if (rtype[j] == 2) c += 1.5;
        if (rtype[j] == 3) c += 6.0;
        return c;
    };
    std::vector<int> order = subset;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    out.n_chunks = int((order.size() + waves - 1) / waves);
    out.recs.assign(size_t(std::max(out.n_chunks, 1)) * waves, RxnRec{});
    for (auto& r : out.recs) {
        std::memset(&r, 0, sizeof(r));
        r.cls = kNoReaction;
    }
    out.slot_of.assign(R, -1);
    out.chunk_of.assign(R, -1);
    out.pd_of_wave.assign(waves, {});
    for (int c = 0; c < out.n_chunks; ++c) {
        std::vector<int> used(waves, 0);
        for (size_t t = size_t(c) * waves; t < std::min(order.size(), size_t(c + 1) * waves); ++t) {
            const int j = order[t];
            const bool is_pd = rtype[j] >= 1;
            int best = -1;
            for (int w = 0; w < waves && best < 0; ++w)
                if (!used[w] && !(is_pd && int(out.pd_of_wave[w].size()) >= pd_cap)) best = w;
            if (best < 0) return fail(PYRO_E_UNSUPPORTED, "too many third-body reactions in a Jacobian row");
            used[best] = 1;
            if (is_pd) out.pd_of_wave[best].push_back(j);
            out.slot_of[j] = best;
            out.chunk_of[j] = c;
            RxnRec& r = out.recs[size_t(c) * waves + best];
            const auto& rj = (*in.reac)[j];
            const auto& pj = (*in.prod)[j];
            r.cls = rtype[j];
            r.rev = (*in.rev)[j];
            r.nr = int(rj.size());
            r.np = int(pj.size());
            for (int q = 0; q < kMaxSide; ++q) {
                r.r[q] = q < r.nr ? rj[q] * row_bytes : 0;
                r.p[q] = q < r.np ? pj[q] * row_bytes : 0;
            }
            r.dnu = (*in.dnu)[j];
            r.prow = j;
            r.pdw = is_pd ? int(out.pd_of_wave[best].size()) - 1 : -1;
            r.fo = (*in.fo_idx)[j];
            r.qoff = best * kTile * 8;
            r.pd = (*in.pd_row)[j];
        }
    }
    out.max_pdw = 0;
    for (auto& p : out.pd_of_wave) out.max_pdw = std::max<int>(out.max_pdw, int(p.size()));
    return PYRO_OK;
}

// Gathering lists of a schedule: per (chunk, wave), kMaxOwn + 1 boundaries
// into the entries that entries(k, chunk, out) appends for owned species k.
template <typename F>
void gather_lists(const HostSched& sc, F entries, std::vector<int32_t>& ptr,
                  std::vector<uint32_t>& ent) {
    ptr.reserve(size_t(std::max(sc.n_chunks, 1)) * sc.waves * (kMaxOwn + 1));
    for (int c = 0; c < std::max(sc.n_chunks, 1); ++c)
        for (int w = 0; w < sc.waves; ++w)
            for (int i = 0; i <= kMaxOwn; ++i) {
                ptr.push_back(int32_t(ent.size()));
                if (i == kMaxOwn || i >= int(sc.own[w].size())) continue;
                entries(sc.own[w][i], c, ent);
            }
    ent.resize(ent.size() + 2, 0u);  // slack: pairwise loops may read one past
}

// Per-wave tables of a schedule: efficiencies by (wave, species, queue slot),
// pd_stride values per species (the kernel instance's bound on a wave's
// third-body reactions, MAXPD), so that the [M] pass of a wave reads one
// species' values with one scalar load; and the owned species.
void wave_tables(const HostSched& sc, const std::vector<double>& eff,
                 const std::vector<int>& pd_row, int S, int pd_stride, std::vector<double>& effw,
                 std::vector<int32_t>& n_pdw, std::vector<int32_t>& own_tab,
                 std::vector<int32_t>& n_own) {
    effw.assign(std::max(size_t(1), size_t(sc.waves) * S * pd_stride), 0.0);
    n_pdw.assign(sc.waves, 0);
    own_tab.assign(size_t(sc.waves) * kMaxOwn, -1);
    n_own.assign(sc.waves, 0);
    for (int w = 0; w < sc.waves; ++w) {
        n_pdw[w] = int(sc.pd_of_wave[w].size());
        for (int i = 0; i < n_pdw[w] && i < pd_stride; ++i) {
            const int row = pd_row[sc.pd_of_wave[w][i]];
            for (int k = 0; k < S; ++k) effw[(size_t(w) * S + k) * pd_stride + i] = eff[size_t(row) * S + k];
        }
        n_own[w] = int(sc.own[w].size());
        for (size_t i = 0; i < sc.own[w].size(); ++i) own_tab[w * kMaxOwn + i] = sc.own[w][i];
    }
}

int load_mechanism(const char* path, pyro_mech** out) {
    std::ifstream in(path, std::ios::binary);
    if (!in) return fail(PYRO_E_IO, std::string("cannot open ") + path);
    std::vector<uint8_t> blob((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
    Parsed f;
    if (int rc = parse(blob, f)) return rc;
    const int S = int(f.S), R = int(f.R), n_fo = int(f.n_fo), n_pd = int(f.n_tb + f.n_fo);

    // ---- reactions: slots, stoichiometry, classes
    std::vector<std::vector<int>> reac(R), prod(R);
    std::vector<int> dnu(R, 0);
    for (int j = 0; j < R; ++j) {
        for (int q = f.rp[j]; q < f.rp[j + 1]; ++q)
            for (int c = 0; c < f.rn[q]; ++c) reac[j].push_back(f.rs[q]);
        for (int q = f.pp[j]; q < f.pp[j + 1]; ++q)
            for (int c = 0; c < f.pn[q]; ++c) prod[j].push_back(f.ps[q]);
        if (reac[j].empty() || prod[j].empty())
            return fail(PYRO_E_FORMAT, "reaction " + std::to_string(j) + " has an empty side");
        if (reac[j].size() > size_t(kMaxSide) || prod[j].size() > size_t(kMaxSide))
            return fail(PYRO_E_UNSUPPORTED, "reaction " + std::to_string(j) +
                        " has more than 3 molecules on one side");
        dnu[j] = int(prod[j].size()) - int(reac[j].size());
    }
    std::vector<int> pd_row(R, -1), fo_idx(R, -1);
    for (int j = 0, i = 0, fi = 0; j < R; ++j) {
        if (f.rtype[j] >= 1) pd_row[j] = i++;
        if (f.rtype[j] >= 2) fo_idx[j] = fi++;
    }
    // net coefficients per (species, reaction)
    std::vector<std::vector<std::pair<int, double>>> by_species(S);
    int nnz_f = 0, nnz_r = 0, nnz_net = 0;
    for (int j = 0; j < R; ++j) {
        std::vector<double> nu(S, 0.0), nf(S, 0.0), nr(S, 0.0);
        for (int k : prod[j]) nu[k] += 1, nr[k] += 1;
        for (int k : reac[j]) nu[k] -= 1, nf[k] += 1;
        for (int k = 0; k < S; ++k) {
            if (nu[k] != 0) by_species[k].push_back({j, nu[k]});
            nnz_f += nf[k] != 0;
            nnz_r += nr[k] != 0;
            nnz_net += nu[k] != 0;
        }
    }

    // ---- LDS fit of the 64-cell tile
    pyro_mech* m = new pyro_mech();
    m->S = S; m->R = R; m->E = int(f.E); m->n_tb = int(f.n_tb); m->n_fo = n_fo;
    m->nnz_f = nnz_f; m->nnz_r = nnz_r; m->nnz_net = nnz_net;
    m->W = f.W;
    m->params.resize(size_t(R + n_fo) * 3);
    std::copy(f.arrh.begin(), f.arrh.end(), m->params.begin());
    std::copy(f.low.begin(), f.low.end(), m->params.begin() + size_t(R) * 3);
    // the reaction-equilibrium variant needs one T_mid per reaction
    m->kc_ok = true;
    for (int j = 0; j < R && m->kc_ok; ++j) {
        const double tm = f.trange[3 * reac[j][0] + 1];
        for (int k : reac[j]) m->kc_ok = m->kc_ok && f.trange[3 * k + 1] == tm;
        for (int k : prod[j]) m->kc_ok = m->kc_ok && f.trange[3 * k + 1] == tm;
    }
    const bool fits_species = production_rates_lds_bytes(m, false) <= 160 * 1024;
    // when the species rows exclude a second workgroup per CU, one workgroup
    // of twice the wavefronts keeps four of them per SIMD
    if (!fits_species) m->fw_waves = 2 * kWaves;
    const bool fits_reaction = m->kc_ok && production_rates_lds_bytes(m, true) <= 160 * 1024;
    if (!fits_species && !fits_reaction) {
        delete m;
        return fail(PYRO_E_UNSUPPORTED, "mechanism too large for the 64-cell LDS tile");
    }
    m->wdot_variant = fits_species ? PYRO_WDOT_SPECIES_EQUILIBRIUM : PYRO_WDOT_REACTION_EQUILIBRIUM;

    // ---- schedules: the forward kernel's (kWaves waves, kRxnPerWave
    // reactions each per chunk) and the reverse sweep's (kVjpWaves, one each)
    std::vector<std::vector<std::array<int, 3>>> part(S);  // species -> (j, nu', nu'')
    for (int j = 0; j < R; ++j) {
        std::vector<int> cf(S, 0), cr(S, 0);
        for (int k : reac[j]) cf[k]++;
        for (int k : prod[j]) cr[k]++;
        for (int k = 0; k < S; ++k)
            if (cf[k] || cr[k]) part[k].push_back({j, cf[k], cr[k]});
    }
    const SchedInput sin{S, R, &f.rtype, &f.rev, &reac, &prod, &dnu, &pd_row, &fo_idx, &by_species};
    // species each kernel's gathering visits per reaction: net coefficient
    // for the forward sums, any participation for the reverse sweep
    std::vector<std::vector<int>> g_net(R), g_part(R);
    for (int k = 0; k < S; ++k) {
        for (auto& e : by_species[k]) g_net[e.first].push_back(k);
        for (auto& e : part[k]) g_part[e[0]].push_back(k);
    }
    HostSched fw, bw;
    // the forward schedule: at most max(8, ceil(S / 8)) species per wave with
    // 8 wavefronts (16 with 16), ownership weighted by issue order as below
    const int fw_cap = m->fw_waves == kWaves ? std::max(8, (S + kWaves - 1) / kWaves) : 16;
    if (int rc = build_schedule(sin, m->fw_waves, kRxnPerWave, fw_cap, kTile * 16, 1.0, g_net, fw)) {
        delete m;
        return rc;
    }
    if (int rc = build_schedule(sin, kVjpWaves, 1, std::max(4, (S + kVjpWaves - 1) / kVjpWaves),
                                kVjpRow, 1.5, g_part, bw)) {
        delete m;
        return rc;
    }
    const int n_chunks = fw.n_chunks;
    const std::vector<RxnRec>& recs = fw.recs;
    m->max_own = fw.max_own;
    m->max_pdw = fw.max_pdw;
    m->vjp_max_own = bw.max_own;
    m->vjp_max_pdw = bw.max_pdw;
    // forward gathering lists: (chunk, wave, owned species) -> (slot, nu).
    // gptr holds, per (chunk, wave), kMaxOwn + 1 boundaries: the entries of
    // owned species i span [gptr[base + i], gptr[base + i + 1]).
    auto top16 = [](double x) {
        uint64_t b;
        std::memcpy(&b, &x, sizeof b);
        return uint32_t(b >> 48);
    };
    std::vector<int32_t> gptr;
    std::vector<GatherEntry> gent;
    gather_lists(fw, [&](int k, int c, std::vector<uint32_t>& out) {
        for (auto& e : by_species[k])
            if (fw.chunk_of[e.first] == c) {
                const uint32_t qoff = uint32_t(fw.slot_of[e.first] * kTile * 8);
                out.push_back(qoff | (uint32_t(uint16_t(int16_t(int(e.second)))) << 16));
            }
    }, gptr, gent);
    // reverse-sweep gathering lists: per participant two words holding the
    // slot and the coefficients nu', -nu'', nu' - nu'' as the upper 16 bits
    // of their doubles; boundaries count words
    std::vector<int32_t> vgptr;
    std::vector<uint32_t> vgent;
    gather_lists(bw, [&](int k, int c, std::vector<uint32_t>& out) {
        for (auto& e : part[k])
            if (bw.chunk_of[e[0]] == c) {
                out.push_back(uint32_t(bw.slot_of[e[0]] * kTile * 8) | (top16(double(e[1])) << 16));
                out.push_back(top16(-double(e[2])) | (top16(double(e[1] - e[2])) << 16));
            }
    }, vgptr, vgent);
    std::vector<double> comp_d(f.comp.begin(), f.comp.end());
    if (comp_d.empty()) comp_d.push_back(0.0);
    std::vector<double> eff_t(size_t(S) * std::max(n_pd, 1), 0.0);
    for (int i = 0; i < n_pd; ++i)
        for (int k = 0; k < S; ++k) eff_t[size_t(k) * std::max(n_pd, 1) + i] = f.eff[size_t(i) * S + k];

    // ---- species tables
    std::vector<SpeciesRec> sp(S);
    std::vector<NewtonSpecies> ns(S);
    std::vector<double> tmid_groups;
    for (int k = 0; k < S; ++k) {
        const double* a = &f.nasa[size_t(k) * 14];
        for (int r = 0; r < 2; ++r) {
            const double* c = a + 7 * r;
            double* g = r == 0 ? sp[k].lo : sp[k].hi;
            g[0] = c[0];
            g[1] = -c[1] / 2.0;
            g[2] = -c[2] / 6.0;
            g[3] = -c[3] / 12.0;
            g[4] = -c[4] / 20.0;
            g[5] = c[5];
            g[6] = -c[6];
            double* nn = r == 0 ? ns[k].lo : ns[k].hi;
            for (int q = 0; q < 6; ++q) nn[q] = c[q];
        }
        sp[k].t_mid = f.trange[3 * k + 1];
        sp[k].inv_w = 1.0 / f.W[k];
        ns[k].inv_w = 1.0 / f.W[k];
        auto it = std::find(tmid_groups.begin(), tmid_groups.end(), sp[k].t_mid);
        if (it == tmid_groups.end()) {
            if (int(tmid_groups.size()) == kMaxTmidGroups) {
                delete m;
                return fail(PYRO_E_UNSUPPORTED, "more than 4 distinct NASA7 T_mid values");
            }
            tmid_groups.push_back(sp[k].t_mid);
            it = tmid_groups.end() - 1;
        }
        ns[k].group = int(it - tmid_groups.begin());
    }
    std::vector<FalloffRec> fr(std::max(n_fo, 1));
    for (auto& x : fr) std::memset(&x, 0, sizeof(x));
    for (int i = 0; i < n_fo; ++i) {
        const double* t = &f.troe[4 * i];
        fr[i].troe = f.rtype[f.fo[i]] == 3;
        fr[i].alpha = t[0];
        fr[i].a3 = fr[i].troe ? -1.0 / t[1] : 0.0;
        fr[i].a1 = fr[i].troe ? -1.0 / t[2] : 0.0;
        fr[i].a2 = -t[3];
    }
    const int s_pad = (S + 7) / 8 * 8;
    std::vector<double> effw, veffw;
    std::vector<int32_t> n_pdw, vn_pdw, own_tab, n_own, vown_tab, vn_own;
    // MAXPD of the kernel instances each schedule runs with
    const int fpd_stride = fw.max_pdw <= 8 ? 8 : 16;
    const int vpd_stride = bw.max_pdw <= 4 ? 4 : bw.max_pdw <= 8 ? 8 : 16;
    wave_tables(fw, f.eff, pd_row, S, fpd_stride, effw, n_pdw, own_tab, n_own);
    wave_tables(bw, f.eff, pd_row, S, vpd_stride, veffw, vn_pdw, vown_tab, vn_own);
    // the reverse sweep's third-body rows per wave, in the order its chunks
    // meet them (one reaction per wave per chunk)
    std::vector<int32_t> vpd_list(size_t(kVjpWaves) * kMaxPd, -1);
    for (int w = 0; w < kVjpWaves; ++w)
        for (size_t i = 0; i < bw.pd_of_wave[w].size(); ++i)
            vpd_list[w * kMaxPd + i] = pd_row[bw.pd_of_wave[w][i]];
    // the reverse sweep's efficiencies by (wave, third-body row, owned
    // species): the MAXOWN values a wave needs for one row are contiguous
    // (MAXOWN = the kernel instance's species-per-wave bound)
    const int own_stride = bw.max_own <= 4 ? 4 : bw.max_own <= 8 ? 8 : 16;
    std::vector<double> veffo(std::max(size_t(1), size_t(kVjpWaves) * n_pd * own_stride), 0.0);
    for (int w = 0; w < kVjpWaves; ++w)
        for (int j = 0; j < n_pd; ++j)
            for (size_t i = 0; i < bw.own[w].size() && i < size_t(own_stride); ++i)
                veffo[(size_t(w) * n_pd + j) * own_stride + i] = f.eff[size_t(j) * S + bw.own[w][i]];
    // the Jacobian rows' schedules and tables, concatenated over the rows;
    // each row shares the reverse sweep's ownership tables (own, n_own,
    // effo) and has its own records, gathering lists, efficiency queue and
    // third-body list
    struct RowOffsets { size_t rxn, gptr, gent, effw, n_pdw, pd_list, pd_rows; int n_chunks, n_pd_rows; };
    std::vector<RowOffsets> row_off(S);
    std::vector<RxnRec> jrecs;
    std::vector<int32_t> jgptr, jn_pdw, jpd_list, jpd_rows;
    std::vector<uint32_t> jgent;
    std::vector<double> jeffw;
    for (int j = 0; j < S; ++j) {
        std::vector<int> subset;
        for (auto& e : by_species[j]) subset.push_back(e.first);
        HostSched rs;
        if (int rc = build_row_schedule(sin, subset, bw.own, kVjpWaves, kVjpRow, vpd_stride, rs)) {
            delete m;
            return rc;
        }
        RowOffsets& o = row_off[j];
        o.n_chunks = rs.n_chunks;
        o.rxn = jrecs.size();
        jrecs.insert(jrecs.end(), rs.recs.begin(), rs.recs.end());
        std::vector<int32_t> gp;
        std::vector<uint32_t> ge;
        gather_lists(rs, [&](int k, int c, std::vector<uint32_t>& out) {
            for (auto& e : part[k])
                if (rs.chunk_of[e[0]] == c) {
                    out.push_back(uint32_t(rs.slot_of[e[0]] * kTile * 8) | (top16(double(e[1])) << 16));
                    out.push_back(top16(-double(e[2])) | (top16(double(e[1] - e[2])) << 16));
                }
        }, gp, ge);
        o.gptr = jgptr.size();
        jgptr.insert(jgptr.end(), gp.begin(), gp.end());
        o.gent = jgent.size();
        jgent.insert(jgent.end(), ge.begin(), ge.end());
        std::vector<double> ew;
        std::vector<int32_t> np, ot, no;
        wave_tables(rs, f.eff, pd_row, S, vpd_stride, ew, np, ot, no);
        o.effw = jeffw.size();
        jeffw.insert(jeffw.end(), ew.begin(), ew.end());
        o.n_pdw = jn_pdw.size();
        jn_pdw.insert(jn_pdw.end(), np.begin(), np.end());
        o.pd_list = jpd_list.size();
        for (int w = 0; w < kVjpWaves; ++w)
            for (int i = 0; i < kMaxPd; ++i)
                jpd_list.push_back(i < int(rs.pd_of_wave[w].size()) ? pd_row[rs.pd_of_wave[w][i]] : -1);
        // the row's third-body rows, ascending (the rows whose M-bar it stages)
        o.pd_rows = jpd_rows.size();
        std::vector<int> rows;
        for (int w = 0; w < kVjpWaves; ++w)
            for (int jr : rs.pd_of_wave[w]) rows.push_back(pd_row[jr]);
        std::sort(rows.begin(), rows.end());
        o.n_pd_rows = int(rows.size());
        jpd_rows.insert(jpd_rows.end(), rows.begin(), rows.end());
    }
    if (jpd_rows.empty()) jpd_rows.push_back(0);
    if (jrecs.empty()) jrecs.push_back(RxnRec{});
    if (jgent.empty()) jgent.push_back(0u);
    std::vector<DevSched> jrows(std::max(S, 1));   // device pointers filled after the allocation

    std::vector<double> params = m->params;
    if (params.empty()) params.push_back(0.0);
    // B fragments of eps^T for the MFMA third-body variant
    const int n_pb = (n_pd + 15) / 16, n_ks = (S + 3) / 4;
    std::vector<double> eps_frag(std::max(size_t(1), size_t(n_pb) * n_ks * 64), 0.0);
    for (int pb = 0; pb < n_pb; ++pb)
        for (int kk = 0; kk < n_ks; ++kk)
            for (int l = 0; l < 64; ++l) {
                const int j = 16 * pb + (l & 15), k = 4 * kk + (l >> 4);
                if (j < n_pd && k < S)
                    eps_frag[(size_t(pb) * n_ks + kk) * 64 + l] = f.eff[size_t(j) * S + k];
            }
    // combined Gibbs coefficients of every reversible reaction, per forward
    // slot: sum_k nu_kj c_k for both ranges, then T_mid (g0/RT is linear in c)
    std::vector<double> rxn_kc(recs.size() * 16, 0.0);
    if (m->kc_ok) {
        for (size_t slot = 0; slot < recs.size(); ++slot) {
            const RxnRec& r = recs[slot];
            if (r.cls == kNoReaction || !r.rev) continue;
            const int j = r.prow;
            double* d = &rxn_kc[slot * 16];
            auto add = [&](int k, double nu) {
                for (int q = 0; q < 7; ++q) {
                    d[q] += nu * sp[k].lo[q];
                    d[7 + q] += nu * sp[k].hi[q];
                }
            };
            for (int k : prod[j]) add(k, 1.0);
            for (int k : reac[j]) add(k, -1.0);
            d[14] = sp[reac[j][0]].t_mid;
        }
    }

    // B fragments of the net coefficients per forward chunk,
    // [chunk][species block][K-step][lane] = nu[16 sb + l%16][slot 4 kk + l/16]
    // (S <= 64 with kWaves wavefronts, S <= 192 with 2 kWaves)
    // (four blocks with kWaves wavefronts, zero beyond S: the kernel then
    // multiplies every block without a test)
    const int cslots = m->fw_waves * kRxnPerWave, nks = cslots / 4;
    const int nsb = m->fw_waves == kWaves ? 4 : (S + 15) / 16;
    const bool nq_table = m->fw_waves == kWaves ? S <= 64 : S <= 192;
    std::vector<double> nu_frag(
        nq_table ? size_t(std::max(n_chunks, 1)) * nsb * nks * 64 : 1, 0.0);
    if (nq_table)
        for (int c = 0; c < n_chunks; ++c)
            for (int slot = 0; slot < cslots; ++slot) {
                const RxnRec& r = recs[size_t(c) * cslots + slot];
                if (r.cls == kNoReaction) continue;
                const int j = r.prow;
                std::vector<int> nu(S, 0);
                for (int k : prod[j]) nu[k] += 1;
                for (int k : reac[j]) nu[k] -= 1;
                const int kk = slot / 4, row = slot % 4;
                for (int k = 0; k < S; ++k) {
                    if (!nu[k]) continue;
                    const int sb = k / 16, l = row * 16 + k % 16;
                    nu_frag[((size_t(c) * nsb + sb) * nks + kk) * 64 + l] = double(nu[k]);
                }
            }

    // B fragments of nu' and nu'' per forward chunk for the log-space form's
    // matrix-core log products, [chunk][side][slot block][K-step][lane] =
    // nu[4 kk + l/16][slot 16 sb + l%16]; built when that form can run
    const int lp_nsb = cslots / 16, lp_nks = (S + 3) / 4;
    const bool lp_table = m->kc_ok;
    std::vector<double> lp_frag(
        lp_table ? size_t(std::max(n_chunks, 1)) * 2 * lp_nsb * lp_nks * 64 : 1, 0.0);
    if (lp_table)
        for (int c = 0; c < n_chunks; ++c)
            for (int slot = 0; slot < cslots; ++slot) {
                const RxnRec& r = recs[size_t(c) * cslots + slot];
                if (r.cls == kNoReaction) continue;
                const int j = r.prow;
                for (int side = 0; side < 2; ++side)
                    for (int k : side == 0 ? reac[j] : prod[j]) {
                        const int kk = k / 4, l = (k % 4) * 16 + slot % 16;
                        lp_frag[((((size_t(c) * 2 + side) * lp_nsb + slot / 16) * lp_nks + kk) * 64) + l] += 1.0;
                    }
            }

    // ---- one device allocation holding every table
    struct Part { const void* src; size_t bytes; size_t off; };
    std::vector<Part> parts = {
        {sp.data(), sp.size() * sizeof(SpeciesRec), 0},
        {recs.data(), recs.size() * sizeof(RxnRec), 0},
        {fr.data(), fr.size() * sizeof(FalloffRec), 0},
        {effw.data(), effw.size() * sizeof(double), 0},
        {n_pdw.data(), n_pdw.size() * sizeof(int32_t), 0},
        {params.data(), params.size() * sizeof(double), 0},
        {own_tab.data(), own_tab.size() * sizeof(int32_t), 0},
        {n_own.data(), n_own.size() * sizeof(int32_t), 0},
        {gptr.data(), gptr.size() * sizeof(int32_t), 0},
        {gent.data(), gent.size() * sizeof(GatherEntry), 0},
        {ns.data(), ns.size() * sizeof(NewtonSpecies), 0},
        {f.W.data(), f.W.size() * sizeof(double), 0},
        {vgptr.data(), vgptr.size() * sizeof(int32_t), 0},
        {vgent.data(), vgent.size() * sizeof(uint32_t), 0},
        {eff_t.data(), eff_t.size() * sizeof(double), 0},
        {bw.recs.data(), bw.recs.size() * sizeof(RxnRec), 0},
        {comp_d.data(), comp_d.size() * sizeof(double), 0},
        {veffw.data(), veffw.size() * sizeof(double), 0},
        {vn_pdw.data(), vn_pdw.size() * sizeof(int32_t), 0},
        {vown_tab.data(), vown_tab.size() * sizeof(int32_t), 0},
        {vn_own.data(), vn_own.size() * sizeof(int32_t), 0},
        {vpd_list.data(), vpd_list.size() * sizeof(int32_t), 0},
        {rxn_kc.data(), rxn_kc.size() * sizeof(double), 0},
        {eps_frag.data(), eps_frag.size() * sizeof(double), 0},
        {veffo.data(), veffo.size() * sizeof(double), 0},
        {nu_frag.data(), nu_frag.size() * sizeof(double), 0},
        {lp_frag.data(), lp_frag.size() * sizeof(double), 0},
        {jrecs.data(), jrecs.size() * sizeof(RxnRec), 0},
        {jgptr.data(), jgptr.size() * sizeof(int32_t), 0},
        {jgent.data(), jgent.size() * sizeof(uint32_t), 0},
        {jeffw.data(), jeffw.size() * sizeof(double), 0},
        {jn_pdw.data(), jn_pdw.size() * sizeof(int32_t), 0},
        {jpd_list.data(), jpd_list.size() * sizeof(int32_t), 0},
        {jrows.data(), jrows.size() * sizeof(DevSched), 0},
        {jpd_rows.data(), jpd_rows.size() * sizeof(int32_t), 0},
    };
    size_t total = 0;
    for (auto& p : parts) {
        p.off = total;
        total = align256(total + p.bytes);
    }
    std::vector<uint8_t> host(total, 0);
    for (auto& p : parts)
        if (p.bytes) std::memcpy(host.data() + p.off, p.src, p.bytes);

    hipError_t err = hipGetDevice(&m->device);
    if (err != hipSuccess) {
        delete m;
        return hip_fail(err, "hipGetDevice");
    }
    err = hipDeviceGetAttribute(&m->n_cu, hipDeviceAttributeMultiprocessorCount, m->device);
    if (err != hipSuccess) {
        delete m;
        return hip_fail(err, "hipDeviceGetAttribute");
    }
    err = hipMalloc(&m->blob, total);
    if (err != hipSuccess) {
        delete m;
        return err == hipErrorOutOfMemory ? fail(PYRO_E_NOMEM, "hipMalloc of the mechanism tables failed")
                                          : hip_fail(err, "hipMalloc");
    }
    m->blob_bytes = total;
    err = hipMemcpy(m->blob, host.data(), total, hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        (void)hipFree(m->blob);
        delete m;
        return hip_fail(err, "hipMemcpy of the mechanism tables");
    }
    const uint8_t* base = static_cast<const uint8_t*>(m->blob);
    DevMech& d = m->dev;
    d.S = S; d.R = R; d.n_pd = n_pd; d.n_fo = n_fo;
    d.n_chunks = n_chunks;
    d.s_pad = s_pad;
    d.n_groups = int(tmid_groups.size());
    for (int g = 0; g < kMaxTmidGroups; ++g)
        d.t_mid_group[g] = g < d.n_groups ? tmid_groups[g] : 0.0;
    d.species = reinterpret_cast<const SpeciesRec*>(base + parts[0].off);
    d.rxn = reinterpret_cast<const RxnRec*>(base + parts[1].off);
    d.falloff = reinterpret_cast<const FalloffRec*>(base + parts[2].off);
    d.effw = reinterpret_cast<const double*>(base + parts[3].off);
    d.n_pdw = reinterpret_cast<const int32_t*>(base + parts[4].off);
    d.params = reinterpret_cast<const double*>(base + parts[5].off);
    d.own = reinterpret_cast<const int32_t*>(base + parts[6].off);
    d.n_own = reinterpret_cast<const int32_t*>(base + parts[7].off);
    d.gptr = reinterpret_cast<const int32_t*>(base + parts[8].off);
    d.gent = reinterpret_cast<const GatherEntry*>(base + parts[9].off);
    d.newton = reinterpret_cast<const NewtonSpecies*>(base + parts[10].off);
    d.w = reinterpret_cast<const double*>(base + parts[11].off);
    d.eff_t = reinterpret_cast<const double*>(base + parts[14].off);
    d.E = int(f.E);
    d.comp = reinterpret_cast<const double*>(base + parts[16].off);
    DevSched& v = d.vjp;
    v.n_chunks = bw.n_chunks;
    v.rxn = reinterpret_cast<const RxnRec*>(base + parts[15].off);
    v.gptr = reinterpret_cast<const int32_t*>(base + parts[12].off);
    v.gent = reinterpret_cast<const uint32_t*>(base + parts[13].off);
    v.effw = reinterpret_cast<const double*>(base + parts[17].off);
    v.n_pdw = reinterpret_cast<const int32_t*>(base + parts[18].off);
    v.own = reinterpret_cast<const int32_t*>(base + parts[19].off);
    v.n_own = reinterpret_cast<const int32_t*>(base + parts[20].off);
    v.pd_list = reinterpret_cast<const int32_t*>(base + parts[21].off);
    d.rxn_kc = reinterpret_cast<const double*>(base + parts[22].off);
    d.eps_frag = reinterpret_cast<const double*>(base + parts[23].off);
    v.effo = reinterpret_cast<const double*>(base + parts[24].off);
    d.nu_frag = reinterpret_cast<const double*>(base + parts[25].off);
    d.lp_frag = reinterpret_cast<const double*>(base + parts[26].off);
    d.lp_nks = lp_table ? lp_nks : 0;
    // the Jacobian rows' schedule descriptors, now that the tables have
    // device addresses, copied into their part of the allocation
    for (int j = 0; j < S; ++j) {
        const RowOffsets& o = row_off[j];
        DevSched& r = jrows[j];
        r = v;
        r.n_chunks = o.n_chunks;
        r.rxn = reinterpret_cast<const RxnRec*>(base + parts[27].off) + o.rxn;
        r.gptr = reinterpret_cast<const int32_t*>(base + parts[28].off) + o.gptr;
        r.gent = reinterpret_cast<const uint32_t*>(base + parts[29].off) + o.gent;
        r.effw = reinterpret_cast<const double*>(base + parts[30].off) + o.effw;
        r.n_pdw = reinterpret_cast<const int32_t*>(base + parts[31].off) + o.n_pdw;
        r.pd_list = reinterpret_cast<const int32_t*>(base + parts[32].off) + o.pd_list;
        r.n_pd_rows = o.n_pd_rows;
        r.pd_rows = reinterpret_cast<const int32_t*>(base + parts[34].off) + o.pd_rows;
    }
    err = hipMemcpy(static_cast<uint8_t*>(m->blob) + parts[33].off, jrows.data(), jrows.size() * sizeof(DevSched),
                    hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        (void)hipFree(m->blob);
        delete m;
        return hip_fail(err, "hipMemcpy of the Jacobian row schedules");
    }
    d.jac_rows = reinterpret_cast<const DevSched*>(base + parts[33].off);
    err = prepare_production_rates(m);
    if (err == hipSuccess) err = prepare_vjp(m);
    if (err != hipSuccess) {
        (void)hipFree(m->blob);
        delete m;
        return hip_fail(err, "hipFuncSetAttribute");
    }
    *out = m;
    return PYRO_OK;
}

}  // namespace pyro
