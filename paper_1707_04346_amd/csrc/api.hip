// api.hip -- the extern "C" boundary declared in include/cisigma.h.
//
// cisigma_init builds, in order: the GAS occupation types of each spin and the
// allowed (alpha type, beta type) blocks (Sec. 3.1), the padded alpha-major and
// beta-major work layouts, the device string / excitation / pair tables
// (tables.hip), and the integral tables the sigma kernels read: (ij|kl) with
// the kl index packed to pairs k >= l (alpha-beta part), and for each spin the
// pair matrix V of the same-spin part (sigma_ss.hip).
// cisigma_apply enqueues: C -> padded copies, sigma_3, sigma_2, sigma_1,
// padded accumulators -> sigma (Eq. 8: sigma = sigma_1 + sigma_2 + sigma_3).
#include <algorithm>
#include <array>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.h"

#define CIS_API extern "C" __attribute__((visibility("default")))

// Scratch of cisigma_apply_noalloc: the sigma workspace (padded layout copies,
// accumulators and materialised same-spin rows) of spaces small enough to fit,
// in a static device array.  Every GPU the library runs on holds its own copy
// until the process ends; host code never passes `scratch` itself to a kernel
// but the device address looked up once per device (noalloc_scratch below).
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

int cis_set_error(cisigma_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

namespace {

const char *status_text(int s) {
    switch (s) {
        case CISIGMA_OK: return "ok";
        case CISIGMA_EINVAL: return "invalid argument";
        case CISIGMA_ENOMEM: return "out of memory";
        case CISIGMA_EDEVICE: return "HIP device error";
        case CISIGMA_ENOCONV: return "Davidson did not converge within max_iter";
        case CISIGMA_EUNSUPPORTED: return "request outside what this build implements";
        default: return "unknown status";
    }
}

int hip_fail(cisigma_ctx *ctx, hipError_t e, const char *where) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return cis_set_error(ctx, CISIGMA_ENOMEM, std::string(where) + ": device out of memory");
    return cis_set_error(ctx, CISIGMA_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_OR_FAIL(ctx, x, where)                     \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
    } while (0)

// device address of `scratch` on device dev, looked up on the first request for
// that device (with it current) and kept; nullptr with *err set on failure
void *noalloc_scratch(int dev, hipError_t *err) {
    static std::mutex mu;
    static std::array<void *, 64> ptr{};
    *err = hipSuccess;
    if (dev < 0 || dev >= int(ptr.size())) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        ptr[dev] = p;
    }
    return ptr[dev];
}

uint64_t binom(int m, int k) {
    if (k < 0 || k > m) return 0;
    uint64_t c = 1;
    for (int i = 0; i < k; ++i) c = c * uint64_t(m - i) / uint64_t(i + 1);
    return c;
}

// all occupation tuples of `nel` electrons over the GAS spaces
void enum_tuples(const std::vector<int> &gn, int nel, int g, std::vector<int> &cur, std::vector<std::vector<int>> &out) {
    if (g == int(gn.size())) {
        if (nel == 0) out.push_back(cur);
        return;
    }
    for (int k = 0; k <= std::min(nel, gn[g]); ++k) {
        cur[g] = k;
        enum_tuples(gn, nel - k, g + 1, cur, out);
    }
}

bool pair_allowed(const cisigma_ctx *c, const int *ta, const int *tb) {
    int cum = 0;
    for (size_t g = 0; g < c->gas_norb.size(); ++g) {
        cum += ta[g] + tb[g];
        if (cum < c->gas_min[g] || cum > c->gas_max[g]) return false;
    }
    return true;
}

template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src) {
    size_t n = src.size() > 0 ? src.size() : 1;
    hipError_t e = hipMalloc(dst, n * sizeof(T));
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

void free_ctx(cisigma_ctx *c) {
    if (!c) return;
    for (int s = 0; s < 2; ++s) {
        auto &T = c->sp[s];
        (void)hipFree(T.d_str); (void)hipFree(T.d_stype); (void)hipFree(T.d_exc); (void)hipFree(T.d_pairs);
        (void)hipFree(T.d_gkey); (void)hipFree(T.d_graw); (void)hipFree(T.d_radix); (void)hipFree(T.d_adiag);
        (void)hipFree(T.d_remap);
        (void)hipFree(T.d_pair_inv); (void)hipFree(T.d_yoff); (void)hipFree(T.d_ycol); (void)hipFree(T.d_klist);
        auto &L = c->pl[s];
        (void)hipFree(L.d_seg); (void)hipFree(L.d_ld); (void)hipFree(L.d_tile_u); (void)hipFree(L.d_tile_c0);
        (void)hipFree(c->d_tstart[s]);
        (void)hipFree(c->d_v64[s]); (void)hipFree(c->d_v32[s]);
        auto &W = c->ws[s];
        (void)hipFree(W.cp); (void)hipFree(W.sp); (void)hipFree(W.ct); (void)hipFree(W.st); (void)hipFree(W.ys);
    }
    (void)hipFree(c->d_rdm);
    cis::drop_graphs(c);
    (void)hipFree(c->d_gp64); (void)hipFree(c->d_gp32); (void)hipFree(c->d_h64); (void)hipFree(c->d_h32);
    (void)hipFree(c->d_jpq);
    (void)hipFree(c->bt.blk); (void)hipFree(c->bt.tb); (void)hipFree(c->bt.tr); (void)hipFree(c->bt.tc);
    (void)hipFree(c->d_pblk); (void)hipFree(c->d_blkoff);
    (void)hipFree(c->plan.d_entries[0]); (void)hipFree(c->plan.d_entries[1]);
    (void)hipFree(c->d_act_start); (void)hipFree(c->d_act_tiles);
    (void)hipFree(c->go.d_slot); (void)hipFree(c->go.d_coff); (void)hipFree(c->go.d_g32); (void)hipFree(c->go.d_g64);
    for (int d = 0; d < 2; ++d) {
        (void)hipFree(c->go.d_act[d]);
        (void)hipFree(c->go.d_units[d]);
        (void)hipFree(c->go.plan[d].d_entries[0]);
        (void)hipFree(c->go.plan[d].d_entries[1]);
    }
    for (auto e : c->prof_events) (void)hipEventDestroy(e);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    delete c;
}

// host-side string index (same contract as the device tables)
int64_t host_string_index(const cisigma_ctx *c, int spin, uint32_t x) {
    const auto &T = c->sp[spin];
    const int G = c->gas.ngas;
    if (__builtin_popcount(x) != T.nel) return -1;
    if (c->n < 32 && (x >> c->n)) return -1;
    uint64_t key = 0;
    for (int g = 0; g < G; ++g) key += uint64_t(__builtin_popcount(x & c->gas.mask[g])) * c->gas.keymul[g];
    auto it = std::lower_bound(T.gkey.begin(), T.gkey.end(), key);
    if (it == T.gkey.end() || *it != key) return -1;
    int t = int(it - T.gkey.begin());
    uint64_t rank = 0, radix = 1;
    for (int g = 0; g < G; ++g) {
        uint32_t sub = (x & c->gas.mask[g]) >> c->gas.first[g];
        uint64_t r = 0;
        int i = 1;
        while (sub) {
            int p = __builtin_ctz(sub);
            r += binom(p, i);
            ++i;
            sub &= sub - 1;
        }
        rank += r * radix;
        radix *= binom(__builtin_popcount(c->gas.mask[g]), T.gtocc[size_t(t) * G + g]);
    }
    const int64_t raw = T.graw[t] + int64_t(rank);
    return c->sym ? T.remap[size_t(raw)] : raw;
}

// Are alpha type ta and beta type tb a block of the space: GAS bounds on their
// occupations and, with spatial symmetry, irreps multiplying to the target?
bool block_allowed(const cisigma_ctx *c, int ta, int tb) {
    const int G = c->gas.ngas;
    if (!pair_allowed(c, &c->sp[0].tocc[size_t(ta) * G], &c->sp[1].tocc[size_t(tb) * G])) return false;
    return !c->sym || (c->sp[0].tirrep[ta] ^ c->sp[1].tirrep[tb]) == c->target;
}

int build_integrals(cisigma_ctx *c) {
    const int n = c->n;
    const size_t n2 = size_t(n) * n;
    c->npair = n * (n + 1) / 2;
    c->nps = n * (n - 1) / 2;
    c->kp = cis::sigma_ab_kp(c->npair);
    const double *g = c->g.data();
    auto G = [&](int p, int q, int r, int s) { return g[((size_t(p) * n + q) * n + r) * n + s]; };
    // (ij|kl), kl packed k >= l, zero padded to kp
    std::vector<double> gp(n2 * c->kp, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k)
                for (int l = 0; l <= k; ++l) gp[(size_t(i) * n + j) * c->kp + cis::pair_ge(k, l)] = G(i, j, k, l);
    std::vector<float> gp32(gp.begin(), gp.end());
    HIP_OR_FAIL(c, upload(&c->d_gp64, gp), "init: integral upload");
    HIP_OR_FAIL(c, upload(&c->d_gp32, gp32), "init: integral upload");
    std::vector<float> h32(c->h.begin(), c->h.end());
    HIP_OR_FAIL(c, upload(&c->d_h64, c->h), "init: integral upload");
    HIP_OR_FAIL(c, upload(&c->d_h32, h32), "init: integral upload");
    std::vector<double> jpq(n2);
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) jpq[size_t(p) * n + q] = G(p, p, q, q);
    HIP_OR_FAIL(c, upload(&c->d_jpq, jpq), "init: integral upload");
    // same-spin pair matrices (absorbing h / (N-1))
    for (int s = 0; s < 2; ++s) {
        int N = c->sp[s].nel;
        if (N < 2 || c->nps == 0) continue;
        const double f = 1.0 / double(N - 1);
        auto Tm = [&](int p, int q, int r, int t) {
            double v = G(p, q, r, t);
            if (r == t) v += f * c->h[size_t(p) * n + q];
            if (p == q) v += f * c->h[size_t(r) * n + t];
            return v;
        };
        std::vector<double> V(size_t(c->nps) * c->nps);
        for (int r = 1; r < n; ++r)
            for (int p = 0; p < r; ++p) {          // creator pair (p < r)
                int P = cis::pair_gt(r, p);
                for (int t = 1; t < n; ++t)
                    for (int q = 0; q < t; ++q) {  // annihilator pair (q < t)
                        int Q = cis::pair_gt(t, q);
                        V[size_t(P) * c->nps + Q] = Tm(p, q, r, t) - Tm(p, t, r, q);
                    }
            }
        std::vector<float> V32(V.begin(), V.end());
        HIP_OR_FAIL(c, upload(&c->d_v64[s], V), "init: pair matrix upload");
        HIP_OR_FAIL(c, upload(&c->d_v32[s], V32), "init: pair matrix upload");
    }
    return CISIGMA_OK;
}

int build_layouts(cisigma_ctx *c) {
    auto &A = c->sp[0], &B = c->sp[1];
    for (int rs = 0; rs < 2; ++rs) {
        auto &L = c->pl[rs];
        const auto &R = c->sp[rs], &O = c->sp[1 - rs];
        L.rs = rs;
        L.ld.assign(O.ntype, 0);
        for (int u = 0; u < O.ntype; ++u) L.ld[u] = (O.tcount[u] + cis::kTileCols - 1) / cis::kTileCols * cis::kTileCols;
        L.seg.assign(size_t(R.ntype) * O.ntype, -1);
        int64_t off = 0;
        for (int t = 0; t < R.ntype; ++t)
            for (int u = 0; u < O.ntype; ++u) {
                int64_t b = rs == 0 ? c->lay.boff[size_t(t) * B.ntype + u] : c->lay.boff[size_t(u) * B.ntype + t];
                if (b < 0) continue;
                L.seg[size_t(t) * O.ntype + u] = off;
                off += int64_t(R.tcount[t]) * L.ld[u];
            }
        L.size = off;
        L.tile_u.clear();
        L.tile_c0.clear();
        for (int u = 0; u < O.ntype; ++u)
            for (int c0 = 0; c0 < L.ld[u]; c0 += cis::kTileCols) {
                L.tile_u.push_back(u);
                L.tile_c0.push_back(c0);
            }
        L.ntiles = int(L.tile_u.size());
        HIP_OR_FAIL(c, upload(&L.d_seg, L.seg), "init: layout upload");
        HIP_OR_FAIL(c, upload(&L.d_ld, L.ld), "init: layout upload");
        HIP_OR_FAIL(c, upload(&L.d_tile_u, L.tile_u), "init: layout upload");
        HIP_OR_FAIL(c, upload(&L.d_tile_c0, L.tile_c0), "init: layout upload");
        HIP_OR_FAIL(c, upload(&c->d_tstart[rs], c->sp[rs].tstart), "init: layout upload");
    }
    // conversion tiles over the caller-layout blocks
    std::vector<cis::BlockDev> blk(c->lay.nblk);
    std::vector<int> tb, tr, tc;
    for (int b = 0; b < c->lay.nblk; ++b) {
        int ta = c->lay.blk_a[b], tbb = c->lay.blk_b[b];
        cis::BlockDev d{};
        d.ta = ta; d.tb = tbb; d.na = A.tcount[ta]; d.nb = B.tcount[tbb];
        d.off = c->lay.blk_off[b];
        d.sega = c->pl[0].seg[size_t(ta) * B.ntype + tbb];
        d.segb = c->pl[1].seg[size_t(tbb) * A.ntype + ta];
        d.lda = c->pl[0].ld[tbb];
        d.ldb = c->pl[1].ld[ta];
        blk[b] = d;
        for (int r0 = 0; r0 < d.na; r0 += 64)
            for (int c0 = 0; c0 < d.nb; c0 += 64) {
                tb.push_back(b); tr.push_back(r0); tc.push_back(c0);
            }
    }
    c->bt.ntiles = int(tb.size());
    // mirror blocks: the alpha and beta tables, the padded layouts and the block
    // set must be mirror images for the M_S = 0 sector
    bool sym = A.nel == B.nel && A.ntype == B.ntype && A.tocc == B.tocc && A.tcount == B.tcount &&
               A.tirrep == B.tirrep && c->pl[0].seg == c->pl[1].seg && c->pl[0].ld == c->pl[1].ld;
    std::vector<int> pblk(c->lay.nblk, -1);
    for (int b = 0; b < c->lay.nblk && sym; ++b)
        for (int b2 = 0; b2 < c->lay.nblk; ++b2)
            if (c->lay.blk_a[b2] == c->lay.blk_b[b] && c->lay.blk_b[b2] == c->lay.blk_a[b]) pblk[b] = b2;
    for (int b = 0; b < c->lay.nblk && sym; ++b) sym = pblk[b] >= 0;
    c->spin_sym = sym;
    if (sym) {
        HIP_OR_FAIL(c, upload(&c->d_pblk, pblk), "init: block upload");
        HIP_OR_FAIL(c, upload(&c->d_blkoff, c->lay.blk_off), "init: block upload");
    }
    HIP_OR_FAIL(c, upload(&c->bt.blk, blk), "init: block upload");
    HIP_OR_FAIL(c, upload(&c->bt.tb, tb), "init: block upload");
    HIP_OR_FAIL(c, upload(&c->bt.tr, tr), "init: block upload");
    HIP_OR_FAIL(c, upload(&c->bt.tc, tc), "init: block upload");
    return CISIGMA_OK;
}

// Active beta tiles of the general sigma_3 kernel.  A workgroup for source
// alpha string Ja (type ta) and an output beta tile of type u does work only
// when some single alpha excitation of Ja lands in a type allowed with u (a
// sigma block to write) and some single beta excitation into u starts from a
// type allowed with ta (a C block to read); a single excitation moves at most
// one electron between GAS spaces.
int build_active_tiles(cisigma_ctx *c) {
    const auto &A = c->sp[0], &B = c->sp[1];
    const int ng = c->gas.ngas;
    const auto &L = c->pl[0];
    auto reach = [&](const cis::SpinTables &S, int t) {
        // types one single excitation can lead to: the same occupations (any irrep
        // with spatial symmetry) or one electron moved between two GAS spaces
        std::vector<int> out;
        for (int u = 0; u < S.ntype; ++u)
            if (std::equal(S.tocc.begin() + size_t(t) * ng, S.tocc.begin() + size_t(t + 1) * ng,
                           S.tocc.begin() + size_t(u) * ng))
                out.push_back(u);
        for (int i = 0; i < ng; ++i)
            for (int j = 0; j < ng; ++j) {
                if (i == j || S.tocc[size_t(t) * ng + i] == 0) continue;
                std::vector<int> occ(S.tocc.begin() + size_t(t) * ng, S.tocc.begin() + size_t(t + 1) * ng);
                --occ[i];
                ++occ[j];
                for (int u = 0; u < S.ntype; ++u)
                    if (std::equal(occ.begin(), occ.end(), S.tocc.begin() + size_t(u) * ng)) out.push_back(u);
            }
        return out;
    };
    auto allowed = [&](int ta, int tb) { return c->lay.boff[size_t(ta) * B.ntype + tb] >= 0; };
    std::vector<int> start{0}, tiles;
    std::vector<std::vector<int>> rb(B.ntype);
    for (int u = 0; u < B.ntype; ++u) rb[u] = reach(B, u);
    for (int ta = 0; ta < A.ntype; ++ta) {
        const auto ra = reach(A, ta);
        std::vector<char> act(B.ntype, 0);
        for (int u = 0; u < B.ntype; ++u) {
            bool out_ok = false, src_ok = false;
            for (int t2 : ra) out_ok = out_ok || allowed(t2, u);
            for (int u2 : rb[u]) src_ok = src_ok || allowed(ta, u2);
            act[u] = out_ok && src_ok;
        }
        for (int t = 0; t < L.ntiles; ++t)
            if (act[L.tile_u[t]]) tiles.push_back(t);
        start.push_back(int(tiles.size()));
        c->act_max = std::max(c->act_max, start.back() - start[start.size() - 2]);
    }
    if (tiles.empty()) tiles.push_back(0);
    HIP_OR_FAIL(c, upload(&c->d_act_start, start), "init: active tiles");
    HIP_OR_FAIL(c, upload(&c->d_act_tiles, tiles), "init: active tiles");
    return CISIGMA_OK;
}

// Scatter plan of the owner-computes sigma_3 kernel (one-block spaces of up
// to 16 orbitals), built on the host from the device beta excitation lists.
// Per 32-column tile of source strings Jb: every contribution (target Ib,
// W element (kl, column), sign) -- the single beta excitations of each Jb and
// the diagonal kk terms of Ib = Jb -- sorted so that equal targets ("groups")
// are contiguous, cut at group boundaries into four wave ranges of at most
// 64*ew entries; lane l of a wave takes entries [l*ew, (l+1)*ew) of its range.
// Words per wave and tile, as the kernel reads them ([q][lane] order):
//   entry   : bits 16..31 the sigma slot the entry's running sum is written to
//             -- the group's target if the entry ends its group, else the
//             lane's discard slot ld + lane -- as a byte offset (FP32) or an
//             element index (FP64); bits 0..15 the W byte offset, its bit 0
//             (always clear) replaced by the sign
//   header  : bit 0 set when the lane's first entry starts a group (or the lane
//             is padding); the rest is the byte offset the carry from earlier
//             lanes is added to (the target of the lane's first group if that
//             group began in an earlier lane and ends in this one, else the
//             discard slot)
// A group may span at most four lanes (the kernel carries partial sums over
// three).  One encoding per element size.  Without a plan (a shape no kernel
// covers) the general kernel runs.
// Where the contributions of one source tile come from and go to.
struct PlanSpec {
    int ntile = 0;                                 // 32-column source tiles
    std::function<int(int, int)> source;           // (tile, column) -> beta string index, -1: none
    std::function<int(int, int)> w_row;            // orbital pair (k >= l) -> W row
    std::function<int(int)> target;                // beta string -> sigma slot, -1: outside (dropped); none: identity
    int nvirt = 0;                                 // sigma slots (targets < nvirt; discard slots nvirt + lane)
    uint32_t unit[2] = {8, 4};                     // bytes per unit of the slot field: [FP64, FP32]
    std::function<int(int)> width;                 // entries per lane the kernel compiles for `need`, 0: none
};

// The contributions of every source tile (target slot, W element, sign),
// sorted by target, with group starts and ends marked, and the smallest entry
// count per lane whose four wave ranges hold every tile.
struct PlanItem { uint32_t tgt, widx, neg, start, end; };
struct PlanTiles {
    std::vector<std::vector<PlanItem>> tiles;
    int need = 1;
};

int plan_items(cisigma_ctx *c, const PlanSpec &ps, const std::vector<uint32_t> &exc, const std::vector<uint32_t> &str,
               PlanTiles &out) {
    constexpr int WS = 33;
    const auto &B = c->sp[1];
    out.tiles.assign(ps.ntile, {});
    out.need = 1;
    for (int t = 0; t < ps.ntile; ++t) {
        auto &tile = out.tiles[t];
        for (int col = 0; col < 32; ++col) {
            const int Jb = ps.source(t, col);
            if (Jb < 0) continue;
            auto push = [&](int Ib, int k, int l, uint32_t neg) {
                const int slot = ps.target ? ps.target(Ib) : Ib;
                if (slot < 0) return;
                tile.push_back({uint32_t(slot), uint32_t(ps.w_row(std::max(k, l), std::min(k, l)) * WS + col), neg, 0u, 0u});
            };
            for (int e = 0; e < B.nexc; ++e) {
                const uint32_t w = exc[size_t(Jb) * B.nexc + e];
                if (w == cis::kExcNone) continue;
                push(int(w >> 11), (w >> 6) & 31, (w >> 1) & 31, w & 1u);
            }
            for (uint32_t b = str[Jb]; b; b &= b - 1) {
                const int k = __builtin_ctz(b);
                push(Jb, k, k, 0u);
            }
        }
        std::stable_sort(tile.begin(), tile.end(), [](const PlanItem &a, const PlanItem &b) { return a.tgt < b.tgt; });
        for (size_t i = 0; i < tile.size(); ++i) {
            tile[i].start = (i == 0 || tile[i].tgt != tile[i - 1].tgt);
            tile[i].end = (i + 1 == tile.size() || tile[i].tgt != tile[i + 1].tgt);
        }
        // smallest ew whose wave capacity 64*ew packs the groups into four ranges
        auto fits = [&](size_t cap) {
            int ranges = 1;
            size_t cur = 0;
            for (size_t i = 0; i < tile.size();) {
                size_t j = i + 1;
                while (j < tile.size() && !tile[j].start) ++j;
                const size_t g = j - i;
                if (g > cap) return false;
                if (cur + g > cap) { ++ranges; cur = 0; }
                cur += g;
                i = j;
            }
            return ranges <= 4;
        };
        while (!fits(size_t(64) * out.need)) ++out.need;
    }
    return CISIGMA_OK;
}

// wave ranges of a tile for entries-per-lane ew; false when a group would
// span more than four lanes
bool plan_ranges(const std::vector<PlanItem> &tile, int ew, std::vector<std::pair<size_t, size_t>> &rg) {
    rg.clear();
    const size_t cap = size_t(64) * ew;
    size_t i = 0;
    for (int wv = 0; wv < 4 && i < tile.size(); ++wv) {
        size_t j = i;
        while (j < tile.size()) {
            size_t g = j + 1;
            while (g < tile.size() && !tile[g].start) ++g;
            if (g - i > cap) break;
            j = g;
        }
        for (size_t g0 = i; g0 < j;) {
            size_t g1 = g0 + 1;
            while (g1 < j && !tile[g1].start) ++g1;
            if ((g1 - 1 - i) / ew - (g0 - i) / ew > 3) return false;
            g0 = g1;
        }
        rg.push_back({i, j});
        i = j;
    }
    return i == tile.size();
}

bool plan_fits(const PlanTiles &pt, int ew) {
    std::vector<std::pair<size_t, size_t>> rg;
    for (const auto &tile : pt.tiles)
        if (!plan_ranges(tile, ew, rg)) return false;
    return true;
}

// plan words of every tile for entry count ew, appended to out[FP64], out[FP32];
// with widths, tile t spreads its entries over widths[t] <= ew entries per lane
// (the remaining words of each lane are padding; the header stays at index ew)
void plan_emit(const PlanSpec &ps, const PlanTiles &pt, int ew, std::vector<uint32_t> (&out)[2],
               const std::vector<int> *widths = nullptr) {
    const size_t per_wave = size_t(ew + 1) * 64, per_tile = 4 * per_wave;
    std::vector<std::pair<size_t, size_t>> rg;
    for (int es_i = 0; es_i < 2; ++es_i) {
        const uint32_t es = es_i == 0 ? 8 : 4;   // [0]: FP64, [1]: FP32
        auto &PL = out[es_i];
        const size_t base0 = PL.size();
        PL.resize(base0 + per_tile * pt.tiles.size());
        for (size_t t = 0; t < pt.tiles.size(); ++t) {
            const auto &tile = pt.tiles[t];
            const int w = widths ? (*widths)[t] : ew;
            plan_ranges(tile, w, rg);
            for (int wv = 0; wv < 4; ++wv) {
                const size_t base = base0 + (t * 4 + wv) * per_wave;
                const size_t i = wv < int(rg.size()) ? rg[wv].first : 0, j = wv < int(rg.size()) ? rg[wv].second : 0;
                for (int lane = 0; lane < 64; ++lane) {
                    const uint32_t spare = (uint32_t(ps.nvirt) + lane) * es;    // discard slot, bytes
                    const uint32_t unit = ps.unit[es_i];                         // slot field unit, bytes
                    uint32_t hdr = spare | 1u;
                    for (int q = 0; q < ew; ++q) {
                        const size_t e = i + size_t(lane) * w + q;
                        // padding: the discard slot, and W element (0, 32) -- the tile's pad
                        // column, which kernels that run padding entries keep at zero (a
                        // padding entry may follow the part of a group that continues in
                        // the next lane, when the tile's width is below ew)
                        uint32_t word = ((spare / unit) << 16) | (32u * es);   // column 32 of the 33-wide W rows
                        if (q < w && e < j) {
                            const PlanItem &it = tile[e];
                            const uint32_t slot = it.end ? it.tgt * es : spare;
                            word = ((slot / unit) << 16) | (it.widx * es) | it.neg;
                            if (q == 0 && !it.start) {
                                // continued group: its end in this lane takes the carry
                                hdr = spare;
                                for (size_t f = e; f < i + size_t(lane + 1) * w && f < j; ++f)
                                    if (tile[f].end) { hdr = tile[f].tgt * es; break; }
                            }
                        }
                        PL[base + size_t(q) * 64 + lane] = word;
                    }
                    PL[base + size_t(ew) * 64 + lane] = hdr;
                }
            }
        }
    }
}

int plan_tables(cisigma_ctx *c, std::vector<uint32_t> &exc, std::vector<uint32_t> &str) {
    const auto &B = c->sp[1];
    exc.resize(size_t(B.nstr) * B.nexc);
    str.resize(B.nstr);
    HIP_OR_FAIL(c, hipMemcpy(exc.data(), B.d_exc, exc.size() * 4, hipMemcpyDeviceToHost), "init: scatter plan");
    HIP_OR_FAIL(c, hipMemcpy(str.data(), B.d_str, str.size() * 4, hipMemcpyDeviceToHost), "init: scatter plan");
    return CISIGMA_OK;
}

// Builds the two encodings of a scatter plan into P (P.ew = 0: no plan).
int make_scatter_plan(cisigma_ctx *c, const PlanSpec &ps, cis::ScatterPlan &P) {
    std::vector<uint32_t> exc, str;
    int rc = plan_tables(c, exc, str);
    if (rc) return rc;
    PlanTiles pt;
    rc = plan_items(c, ps, exc, str, pt);
    if (rc) return rc;
    int ew = 0;
    for (int cand : {ps.width(pt.need), 16})
        if (cand >= pt.need && ps.width(cand) == cand && plan_fits(pt, cand)) { ew = cand; break; }
    if (ew == 0) return CISIGMA_OK;
    std::vector<uint32_t> plan[2];
    plan_emit(ps, pt, ew, plan);
    HIP_OR_FAIL(c, upload(&P.d_entries[0], plan[0]), "init: scatter plan");
    HIP_OR_FAIL(c, upload(&P.d_entries[1], plan[1]), "init: scatter plan");
    P.ntile = ps.ntile;
    P.ew = ew;
    return CISIGMA_OK;
}

int build_scatter_plan(cisigma_ctx *c) {
    constexpr int WS = 33;
    const auto &B = c->sp[1];
    const int ld = c->pl[0].ld[0];
    const int mp = 16 * ((c->npair + 15) / 16);
    // 16-bit fields: W byte offsets (FP64 the larger) and slot offsets (FP32 bytes, FP64 elements)
    if (!c->cas || c->n > 16 || B.nexc == 0 || c->na == 0 || size_t(mp) * WS * 8 >= 65536 ||
        (size_t(ld) + 64) * 4 >= 65536)
        return CISIGMA_OK;
    PlanSpec ps;
    ps.ntile = ld / 32;
    ps.source = [&](int t, int col) { const int Jb = t * 32 + col; return Jb < B.nstr ? Jb : -1; };
    ps.w_row = [](int k, int l) { return cis::pair_ge(k, l); };
    ps.nvirt = ld;
    ps.unit[0] = 8;
    ps.unit[1] = 1;
    const int anexc = c->sp[0].nexc, npair = c->npair;
    ps.width = [=](int need) { return cis::sigma_ab_owner_width(anexc, npair, need); };
    return make_scatter_plan(c, ps, c->plan);
}


// Tables of the owner-computes sigma_3 kernel for GAS spaces (see GasOwner):
// W rows = orbital pairs k >= l ordered by the GAS spaces of k and l; the
// gathered rows of an alpha string of type ta = its single excitations ordered
// by source type (the source type of an excitation depends only on ta, since
// spaces are contiguous orbital ranges), then the string itself; per alpha type
// the 32-column source tiles (one beta type each) with the k steps whose
// gathered rows have a block with that beta type.  Per unit (alpha type x
// column range that fits the LDS) the tiles that reach the range, each with the
// 16-row W blocks its plan entries read.  Without a compiled kernel for the
// shape (or when the tables do not fit) the general kernel runs.
//
// One-block spaces come here when their sigma row is too long for the one-block
// kernel (or on request, CISIGMA_OPT_SIGMA_PATH = 2).  Their units split the row
// at the occupations of the two highest orbitals t1 = n-2 < t2 = n-1: in colex
// order the strings with a given occupation of (t2, t1) are one contiguous
// range.  A single excitation E_kl keeps both occupations unless k or l is t1
// or t2, so the W rows are grouped, each group on whole 16-row blocks, as
//   pairs that keep both (k, l < t1; (t1,t1), (t2,t2); and (t2,t1), which
//   only swaps an electron between t1 and t2), then (t1, l < t1), then
//   (t2, l < t1),
// and a source tile of another class than the unit's multiplies only the
// blocks that lead into it (one or two instead of all).
int build_gas_owner(cisigma_ctx *c, bool one_block) {
    constexpr int WS = 33;
    auto &G = c->go;
    const auto &A = c->sp[0], &B = c->sp[1];
    const int n = c->n, ng = c->gas.ngas;
    // one-block spaces come here only when the one-block owner kernel has no plan
    // (more than 16 orbitals, or a sigma row longer than its LDS), or on request
    if ((c->cas && c->plan.ew > 0 && !one_block) || c->na == 0 || c->nb == 0 || A.nexc == 0 || B.nexc == 0)
        return CISIGMA_OK;
    std::vector<int> space(n, 0);
    for (int g = 0; g < ng; ++g)
        for (int o = 0; o < n; ++o)
            if ((c->gas.mask[g] >> o) & 1u) space[o] = g;
    std::vector<std::pair<int, int>> pairs;
    for (int k = 0; k < n; ++k)
        for (int l = 0; l <= k; ++l) pairs.push_back({k, l});
    std::vector<int> row_of(c->npair);
    int nrows = 0;
    const bool classes = c->cas && n >= 3;
    if (classes) {
        const int t1 = n - 2, t2 = n - 1;
        auto group = [&](int k, int l) { return k < t1 || k == l || (k == t2 && l == t1) ? 0 : k == t1 ? 1 : 2; };
        for (int g = 0; g < 3; ++g) {
            for (const auto &pr : pairs)
                if (group(pr.first, pr.second) == g) row_of[cis::pair_ge(pr.first, pr.second)] = nrows++;
            nrows = (nrows + 15) / 16 * 16;
        }
        // Placement for the eight-wave unit kernel, whose producing waves take three
        // runs of w = ceil(blocks / 3) row blocks: the (t2, l) block ends the first
        // run, the (t1, l) block ends the last, and (t2, t1) takes the last row of the
        // second run, so that a source tile of the other t2 class (it needs only the
        // (t2, l) block and (t2, t1)) keeps two SIMDs busy instead of one.
        const int nb = nrows / 16, w = (nb + 2) / 3;
        if (t1 <= 16 && nb >= 6 && 2 * w - 1 < nb - 1) {
            std::vector<int> inner_rows;   // rows of the inner blocks in order, the swap slot held back
            const int b17 = w - 1, b16 = nb - 1, bsw = 2 * w - 1;
            for (int b = 0; b < nb; ++b)
                if (b != b17 && b != b16)
                    for (int r = 0; r < 16; ++r)
                        if (!(b == bsw && r == 15)) inner_rows.push_back(16 * b + r);
            size_t q = 0;
            int r16 = 16 * b16, r17 = 16 * b17;
            bool fits = true;
            for (const auto &pr : pairs) {
                const int k = pr.first, l = pr.second, idx = cis::pair_ge(k, l);
                if (k == t2 && l == t1) row_of[idx] = 16 * bsw + 15;
                else if (group(k, l) == 0) { if (q < inner_rows.size()) row_of[idx] = inner_rows[q++]; else fits = false; }
                else if (group(k, l) == 1) row_of[idx] = r16++;
                else row_of[idx] = r17++;
            }
            if (!fits || r16 > 16 * b16 + 16 || r17 > 16 * b17 + 16) {   // back to the grouped order
                nrows = 0;
                for (int g = 0; g < 3; ++g) {
                    for (const auto &pr : pairs)
                        if (group(pr.first, pr.second) == g) row_of[cis::pair_ge(pr.first, pr.second)] = nrows++;
                    nrows = (nrows + 15) / 16 * 16;
                }
            }
        }
    } else {
        std::stable_sort(pairs.begin(), pairs.end(), [&](const std::pair<int, int> &x, const std::pair<int, int> &y) {
            return std::make_pair(space[x.first], space[x.second]) < std::make_pair(space[y.first], space[y.second]);
        });
        for (int r = 0; r < c->npair; ++r) row_of[cis::pair_ge(pairs[r].first, pairs[r].second)] = r;
        nrows = c->npair;
    }
    const int rb = (nrows + 15) / 16, mp = 16 * rb;
    const int ks = (A.nexc + 1 + 3) / 4, kp = 4 * ks;
    if (ks > 32 || rb > 32 || B.ntype > 255 || size_t(mp) * WS * 8 >= 65536) return CISIGMA_OK;
    if (cis::sigma_ab_gas_width(ks, rb, 1) == 0) return CISIGMA_OK;
    // type moved by one electron from space `from` to space `to` (-1: no such type)
    auto moved = [&](const cis::SpinTables &S, int t, int from, int to) {
        if (from == to) return t;
        std::vector<int> occ(S.tocc.begin() + size_t(t) * ng, S.tocc.begin() + size_t(t + 1) * ng);
        if (occ[from] == 0) return -1;
        --occ[from];
        ++occ[to];
        for (int u = 0; u < S.ntype; ++u)
            if (std::equal(occ.begin(), occ.end(), S.tocc.begin() + size_t(u) * ng)) return u;
        return -1;
    };
    auto allowed = [&](int ta, int tb) { return ta >= 0 && tb >= 0 && c->lay.boff[size_t(ta) * B.ntype + tb] >= 0; };
    std::vector<int> gsize(ng, 0);
    for (int o = 0; o < n; ++o) ++gsize[space[o]];
    // gathered-row slots of each alpha type.  With spatial symmetry the source type
    // of an excitation depends on its orbitals' irreps, not on the type alone: the
    // slots then follow the excitation list (source "any", -3), the k-step masks
    // here take every step (the kernel narrows them per beta type from the row
    // offsets of its string), and the tiles and row blocks come from the plans.
    std::vector<int> slot(size_t(A.ntype) * kp, -1), slot_src(size_t(A.ntype) * kp, -1);
    for (int ta = 0; ta < A.ntype && c->sym; ++ta) {
        for (int q = 0; q < A.nexc; ++q) {
            slot[size_t(ta) * kp + q] = q;
            slot_src[size_t(ta) * kp + q] = -3;
        }
        slot[size_t(ta) * kp + A.nexc] = -2;
        slot_src[size_t(ta) * kp + A.nexc] = ta;
    }
    for (int ta = 0; ta < A.ntype && !c->sym; ++ta) {
        std::vector<int> occ_space, vir_space;   // GAS space of the i-th occupied / virtual orbital
        for (int g = 0; g < ng; ++g) {
            const int occ = A.tocc[size_t(ta) * ng + g];
            for (int q = 0; q < occ; ++q) occ_space.push_back(g);
            for (int q = occ; q < gsize[g]; ++q) vir_space.push_back(g);
        }
        std::vector<std::pair<int, int>> es;   // (source type, excitation index)
        for (int io = 0; io < c->na; ++io)
            for (int iv = 0; iv < n - c->na; ++iv)
                es.push_back({moved(A, ta, occ_space[io], vir_space[iv]), io * (n - c->na) + iv});
        es.push_back({ta, -2});
        std::stable_sort(es.begin(), es.end(), [](const std::pair<int, int> &x, const std::pair<int, int> &y) {
            return unsigned(x.first) < unsigned(y.first);   // no source type (-1) last
        });
        for (size_t q = 0; q < es.size(); ++q) {
            slot[size_t(ta) * kp + q] = es[q].first >= 0 ? es[q].second : -1;
            slot_src[size_t(ta) * kp + q] = es[q].first;
        }
    }
    // source tiles: 32 columns of one beta type
    std::vector<int> tu, tc;
    for (int u = 0; u < B.ntype; ++u)
        for (int c0 = 0; c0 < B.tcount[u]; c0 += 32) { tu.push_back(u); tc.push_back(c0); }
    // compact columns: the beta types allowed with each alpha type, concatenated
    std::vector<int> coff(size_t(A.ntype) * B.ntype, -1), ncols(A.ntype, 0), btype(B.nstr);
    for (int u = 0; u < B.ntype; ++u)
        for (int i = B.tstart[u]; i < B.tstart[u + 1]; ++i) btype[i] = u;
    for (int ta = 0; ta < A.ntype; ++ta)
        for (int u = 0; u < B.ntype; ++u)
            if (allowed(ta, u)) {
                coff[size_t(ta) * B.ntype + u] = ncols[ta];
                ncols[ta] += B.tcount[u];
            }
    // per alpha type, the source tiles that can change its sigma, with k-step and row-block masks
    std::vector<std::vector<std::array<uint32_t, 4>>> tact(A.ntype);
    for (int ta = 0; ta < A.ntype; ++ta) {
        std::vector<uint32_t> kmask(B.ntype, 0), rmask(B.ntype, 0);
        for (int u2 = 0; u2 < B.ntype; ++u2) {
            for (int q = 0; q < kp; ++q) {
                const int src = slot_src[size_t(ta) * kp + q];
                if (src == -3 || allowed(src, u2)) kmask[u2] |= 1u << (q / 4);
            }
            if (c->sym) {
                rmask[u2] = rb >= 32 ? 0xffffffffu : (1u << rb) - 1u;   // narrowed per tile by the plans
                continue;
            }
            for (const auto &pr : pairs) {
                const int sk = space[pr.first], sl = space[pr.second];
                // E_kl or E_lk on a source of type u2 moves one electron between the two spaces
                if (allowed(ta, moved(B, u2, sl, sk)) || allowed(ta, moved(B, u2, sk, sl)))
                    rmask[u2] |= 1u << (row_of[cis::pair_ge(pr.first, pr.second)] / 16);
            }
        }
        for (size_t t = 0; t < tu.size(); ++t)
            if (kmask[tu[t]] && rmask[tu[t]])
                tact[ta].push_back({uint32_t(t), kmask[tu[t]], rmask[tu[t]], uint32_t(tu[t]) | (uint32_t(tc[t]) << 8)});
    }
    // (ij|kl) with kl in the grouped row order
    std::vector<double> g64(size_t(n) * n * mp, 0.0);
    std::vector<float> g32(g64.size(), 0.0f);
    for (int ij = 0; ij < n * n; ++ij)
        for (const auto &pr : pairs) {
            const int r = row_of[cis::pair_ge(pr.first, pr.second)];
            const double v = c->g[(size_t(ij) * n + pr.first) * n + pr.second];
            g64[size_t(ij) * mp + r] = v;
            g32[size_t(ij) * mp + r] = float(v);
        }
    std::vector<uint32_t> exc, str;
    int rc = plan_tables(c, exc, str);
    if (rc) return rc;
    // per precision: units (alpha type x compact column range that fits the LDS),
    // their plans (targets outside the range dropped) and tile lists without
    // the tiles that reach no column of the range
    const int ntb = B.ntype;
    int64_t ldmax = 0;
    for (int v : c->pl[0].ld) ldmax = std::max<int64_t>(ldmax, v);
    // where units may end: the ends of the beta types (GAS; in compact columns per
    // alpha type) or of the top-orbital classes (one-block), cut further only
    // where a piece alone is longer than a unit may be
    std::vector<int> class_end;
    if (classes) {
        auto cls = [&](int Jb) { return int((str[Jb] >> (n - 2)) & 3u); };
        for (int Jb = 1; Jb <= B.nstr; ++Jb) {
            if (Jb < B.nstr && cls(Jb) < cls(Jb - 1)) { class_end.clear(); break; }   // not colex: plain cuts
            if (Jb == B.nstr || cls(Jb) != cls(Jb - 1)) class_end.push_back(Jb);
        }
    }
    auto cuts_of = [&](int ta, int cap) {
        std::vector<int> ends;
        if (classes) {
            ends = class_end;
        } else {
            for (int u = 0; u < ntb; ++u)
                if (coff[size_t(ta) * ntb + u] >= 0) ends.push_back(coff[size_t(ta) * ntb + u] + B.tcount[u]);
        }
        if (ends.empty() || ends.back() != ncols[ta]) ends = {ncols[ta]};
        std::vector<int> cut{0};
        int lo = 0, hi = 0;
        for (int e : ends) {
            if (e - lo <= cap) { hi = e; continue; }
            if (hi > lo) { cut.push_back(hi); lo = hi; }
            while (e - lo > cap) { lo += cap; cut.push_back(lo); }
            hi = e;
        }
        if (hi > lo) cut.push_back(hi);
        return cut;
    };
    for (int d = 0; d < 2; ++d) {
        const size_t es = d == 0 ? 8 : 4;
        // the kernel addresses C with 32-bit element offsets (its zero row included)
        if (uint64_t(c->pl[0].size) + uint64_t(ldmax) >= (uint64_t(1) << 32)) continue;
        // (point-group spaces: one more word per beta type, the kernel's per-type k-step masks)
        const size_t fixed = (size_t(16) * rb * WS + 64) * es + size_t(4) * (kp + (c->sym ? 1 : 0)) * ntb;
        if (fixed >= 160 * 1024) continue;
        int cmax = int(std::min<size_t>((160 * 1024 - fixed) / es, 65536 - 64 - 1));
        if (c->unit_cols > 0) cmax = std::min(cmax, c->unit_cols);
        std::vector<cis::GasUnit> units;
        std::vector<PlanSpec> specs;
        std::vector<PlanTiles> pts;
        std::vector<std::vector<std::array<uint32_t, 4>>> uact;
        int need = 1;
        for (int ta = 0; ta < A.ntype; ++ta) {
            if (tact[ta].empty() || A.tcount[ta] == 0) continue;
            const std::vector<int> cut = cuts_of(ta, cmax);
            for (size_t ci = 0; ci + 1 < cut.size(); ++ci) {
                const int lo = cut[ci], hi = cut[ci + 1];
                const auto &ta_tiles = tact[ta];
                PlanSpec ps;
                ps.ntile = int(ta_tiles.size());
                ps.source = [&, ta](int t, int col) {
                    const int u = int(ta_tiles[t][3] & 255u), cc = int(ta_tiles[t][3] >> 8) + col;
                    return cc < B.tcount[u] ? B.tstart[u] + cc : -1;
                };
                ps.w_row = [&](int k, int l) { return row_of[cis::pair_ge(k, l)]; };
                ps.target = [&, ta, lo, hi](int Ib) {
                    const int u = btype[Ib], o = coff[size_t(ta) * ntb + u];
                    if (o < 0) return -1;
                    const int x = o + (Ib - B.tstart[u]);
                    return x >= lo && x < hi ? x - lo : -1;
                };
                ps.nvirt = hi - lo;
                ps.unit[0] = 8;
                ps.unit[1] = 4;
                PlanTiles pt;
                rc = plan_items(c, ps, exc, str, pt);
                if (rc) return rc;
                // keep the tiles with at least one target in the range, each with the
                // W row blocks its entries read (the only ones it multiplies)
                std::vector<std::array<uint32_t, 4>> keep;
                PlanTiles kept;
                for (size_t t = 0; t < pt.tiles.size(); ++t)
                    if (!pt.tiles[t].empty()) {
                        uint32_t used = 0;
                        for (const auto &it : pt.tiles[t]) used |= 1u << (it.widx / WS / 16);
                        keep.push_back(ta_tiles[t]);
                        keep.back()[2] = used;
                        kept.tiles.push_back(std::move(pt.tiles[t]));
                    }
                if (keep.empty()) continue;
                need = std::max(need, pt.need);
                cis::GasUnit gu;
                gu.ta = ta;
                gu.lo = lo;
                gu.hi = hi;
                units.push_back(gu);
                specs.push_back(ps);
                pts.push_back(std::move(kept));
                uact.push_back(std::move(keep));
            }
        }
        if (units.empty()) continue;
        // splitting rows repeats the gathers of every tile that reaches several
        // units, and its products where they lead into several: give the
        // precision to the general kernel when the row-block products more than
        // double
        {
            double split = 0, whole = 0;
            for (size_t k = 0; k < units.size(); ++k)
                for (const auto &e : uact[k]) split += double(__builtin_popcount(e[2])) * A.tcount[units[k].ta];
            for (int ta = 0; ta < A.ntype; ++ta)
                for (const auto &e : tact[ta]) whole += double(__builtin_popcount(e[2])) * A.tcount[ta];
            if (split > 2.0 * whole) continue;
        }
        // longest rows of work first (one launch covers every unit; the longest workgroups start first)
        {
            std::vector<size_t> ord(units.size());
            for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
            std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return uact[x].size() > uact[y].size(); });
            std::vector<cis::GasUnit> u2;
            std::vector<PlanSpec> s2;
            std::vector<PlanTiles> p2;
            std::vector<std::vector<std::array<uint32_t, 4>>> a2;
            for (size_t k : ord) {
                u2.push_back(units[k]);
                s2.push_back(specs[k]);
                p2.push_back(std::move(pts[k]));
                a2.push_back(std::move(uact[k]));
            }
            units.swap(u2);
            specs.swap(s2);
            pts.swap(p2);
            uact.swap(a2);
        }
        int ew = 0;
        for (int cand : {cis::sigma_ab_gas_width(ks, rb, need), 16}) {
            if (cand < need || cis::sigma_ab_gas_width(ks, rb, cand) != cand) continue;
            bool ok = true;
            for (size_t k = 0; k < pts.size() && ok; ++k) ok = plan_fits(pts[k], cand);
            if (ok) { ew = cand; break; }
        }
        if (ew == 0) continue;
        std::vector<uint32_t> plan[2], act;
        int tile0 = 0;
        std::vector<std::pair<size_t, size_t>> rgw;
        for (size_t k = 0; k < units.size(); ++k) {
            // each tile at the fewest entries per lane that hold it (the kernel reads no more)
            std::vector<int> widths(pts[k].tiles.size(), ew);
            for (size_t t = 0; t < widths.size(); ++t)
                for (int w = 1; w < ew; ++w)
                    if (plan_ranges(pts[k].tiles[t], w, rgw)) { widths[t] = w; break; }
            plan_emit(specs[k], pts[k], ew, plan, &widths);
            units[k].act0 = int(act.size() / 4);
            units[k].nact = int(uact[k].size());
            for (size_t t = 0; t < uact[k].size(); ++t) {
                act.push_back(uint32_t(tile0 + int(t)) | (uint32_t(widths[t]) << 24));
                act.push_back(uact[k][t][1]);
                act.push_back(uact[k][t][2]);
                act.push_back(uact[k][t][3]);
            }
            tile0 += int(uact[k].size());
        }
        if (size_t(tile0) * 4 * (ew + 1) * 64 * 4 >= (size_t(1) << 31)) continue;
        std::vector<int> utab;
        int nblk = 0, maxc = 0;
        G.launch[d].clear();
        for (const auto &un : units) {
            utab.insert(utab.end(), {un.ta, un.lo, un.hi, un.act0, un.nact, A.tstart[un.ta], nblk, 0});
            G.launch[d].push_back({nblk, A.tcount[un.ta]});
            nblk += A.tcount[un.ta];
            maxc = std::max(maxc, un.hi - un.lo);
        }
        HIP_OR_FAIL(c, upload(&G.plan[d].d_entries[d], plan[d]), "init: GAS owner tables");
        HIP_OR_FAIL(c, upload(&G.d_act[d], act), "init: GAS owner tables");
        HIP_OR_FAIL(c, upload(&G.d_units[d], utab), "init: GAS owner tables");
        G.nblocks[d] = nblk;
        G.maxcols[d] = maxc;
        G.plan[d].ntile = tile0;
        G.plan[d].ew = ew;
        G.units[d] = std::move(units);
    }
    if (G.units[0].empty() && G.units[1].empty()) return CISIGMA_OK;
    HIP_OR_FAIL(c, upload(&G.d_slot, slot), "init: GAS owner tables");
    HIP_OR_FAIL(c, upload(&G.d_coff, coff), "init: GAS owner tables");
    HIP_OR_FAIL(c, upload(&G.d_g64, g64), "init: GAS owner tables");
    HIP_OR_FAIL(c, upload(&G.d_g32, g32), "init: GAS owner tables");
    G.ks = ks;
    G.rb = rb;
    return CISIGMA_OK;
}

// Same-spin tables of spaces with several types (GAS occupation types or
// irreps).  (1) Pair lists: many entries of a K lead out of the space (GAS
// bounds, irreps), so each K's entries in the space are moved to the front of
// its list (the inverse table follows) and the K are grouped by that count
// into buckets, each launched with the smallest compiled pair-kernel shape that
// holds its count.  (2) Rows of the materialised products: the product row of
// pair entry (K, e) is the padded sigma row of the string J = K + e, so the
// gather of string I sums the rows of its occupied pairs element by element, as
// for one-block spaces; rows follow the entries in (K, e) order.  Only when
// every spin with pairs has at most 64 occupied pairs per string; otherwise
// the same-spin parts stay on the atomic kernels.
int build_same_spin_rows(cisigma_ctx *c) {
    if (c->cas) return CISIGMA_OK;
    for (int s = 0; s < 2; ++s) {
        auto &S = c->sp[s];
        if (S.nel < 2 || S.nstr == 0 || S.nK == 0 || !S.d_pairs) continue;
        std::vector<uint32_t> pairs(size_t(S.nK) * S.npv);
        HIP_OR_FAIL(c, hipMemcpy(pairs.data(), S.d_pairs, pairs.size() * 4, hipMemcpyDeviceToHost), "init: pair lists");
        std::vector<int> newpos(pairs.size()), count(S.nK, 0);
        for (int K = 0; K < S.nK; ++K) {
            uint32_t *row = pairs.data() + size_t(K) * S.npv;
            int *np = newpos.data() + size_t(K) * S.npv;
            std::vector<uint32_t> in, out;
            for (int e = 0; e < S.npv; ++e) {
                if (row[e] != cis::kPairNone) { np[e] = int(in.size()); in.push_back(row[e]); }
            }
            count[K] = int(in.size());
            int q = count[K];
            for (int e = 0; e < S.npv; ++e)
                if (row[e] == cis::kPairNone) np[e] = q++;
            for (int e = 0; e < S.npv; ++e) row[e] = e < count[K] ? in[e] : cis::kPairNone;
        }
        // buckets: K ordered by the shape that holds its count
        std::vector<std::pair<int, int>> shape_of(S.nK, {-1, -1});
        bool ok = true;
        for (int K = 0; K < S.nK && ok; ++K)
            if (count[K] > 0) ok = cis::same_spin_shape_for(count[K], &shape_of[K].first, &shape_of[K].second);
        if (!ok) continue;   // keep the plain lists
        HIP_OR_FAIL(c, hipMemcpy(S.d_pairs, pairs.data(), pairs.size() * 4, hipMemcpyHostToDevice), "init: pair lists");
        if (S.d_pair_inv) {
            const size_t per = size_t(S.nel) * (S.nel - 1) / 2;
            std::vector<int> inv(size_t(S.nstr) * per);
            HIP_OR_FAIL(c, hipMemcpy(inv.data(), S.d_pair_inv, inv.size() * 4, hipMemcpyDeviceToHost), "init: pair lists");
            for (int &v : inv)
                if (v >= 0) v = (v / S.npv) * S.npv + newpos[size_t(v)];
            HIP_OR_FAIL(c, hipMemcpy(S.d_pair_inv, inv.data(), inv.size() * 4, hipMemcpyHostToDevice), "init: pair lists");
        }
        std::vector<std::pair<int, int>> shapes;
        for (int K = 0; K < S.nK; ++K)
            if (count[K] > 0 && std::find(shapes.begin(), shapes.end(), shape_of[K]) == shapes.end())
                shapes.push_back(shape_of[K]);
        std::sort(shapes.begin(), shapes.end(), [](const std::pair<int, int> &x, const std::pair<int, int> &y) {
            return 16 * x.second * 4 * x.first > 16 * y.second * 4 * y.first;   // heaviest buckets first
        });
        std::vector<int> klist;
        S.bk_ks.clear(); S.bk_mbl.clear(); S.bk_start.assign(1, 0);
        for (const auto &sh : shapes) {
            for (int K = 0; K < S.nK; ++K)
                if (count[K] > 0 && shape_of[K] == sh) klist.push_back(K);
            S.bk_ks.push_back(sh.first);
            S.bk_mbl.push_back(sh.second);
            S.bk_start.push_back(int(klist.size()));
        }
        if (klist.empty()) klist.push_back(0);
        HIP_OR_FAIL(c, upload(&S.d_klist, klist), "init: pair lists");
    }
    for (int s = 0; s < 2; ++s) {
        const auto &S = c->sp[s];
        if (S.nel < 2 || S.nstr == 0) continue;
        if (S.nel * (S.nel - 1) / 2 > 64 || !S.d_pair_inv || !S.d_pairs || !S.d_klist) return CISIGMA_OK;
    }
    for (int s = 0; s < 2; ++s) {
        auto &S = c->sp[s];
        if (S.nel < 2 || S.nstr == 0) continue;
        const auto &L = c->pl[s];
        const int nto = c->sp[1 - s].ntype;
        std::vector<int> ycol(size_t(S.ntype) * nto, -1);
        std::vector<int64_t> rowlen(S.ntype, 0);
        for (int t = 0; t < S.ntype; ++t)
            for (int u = 0; u < nto; ++u)
                if (L.seg[size_t(t) * nto + u] >= 0) {
                    ycol[size_t(t) * nto + u] = int(rowlen[t]);
                    rowlen[t] += L.ld[u];
                }
        std::vector<uint32_t> pairs(size_t(S.nK) * S.npv);
        std::vector<int> stype(S.nstr);
        HIP_OR_FAIL(c, hipMemcpy(pairs.data(), S.d_pairs, pairs.size() * 4, hipMemcpyDeviceToHost), "init: same-spin rows");
        HIP_OR_FAIL(c, hipMemcpy(stype.data(), S.d_stype, stype.size() * 4, hipMemcpyDeviceToHost), "init: same-spin rows");
        std::vector<int64_t> yoff(pairs.size(), -1);
        int64_t tot = 0;
        for (size_t i = 0; i < pairs.size(); ++i) {
            if (pairs[i] == cis::kPairNone) continue;
            yoff[i] = tot;
            tot += rowlen[stype[pairs[i] >> 11]];
        }
        HIP_OR_FAIL(c, upload(&S.d_yoff, yoff), "init: same-spin rows");
        HIP_OR_FAIL(c, upload(&S.d_ycol, ycol), "init: same-spin rows");
        S.ny = tot;
    }
    return CISIGMA_OK;
}

// elements of the materialised same-spin rows of a space with several types
// (the larger spin; the passes reuse one buffer), 0: none
int64_t ys_rows_elems(const cisigma_ctx *c) {
    if (c->cas) return 0;
    int64_t m = 0;
    for (int s = 0; s < 2; ++s) {
        const auto &S = c->sp[s];
        if (S.nel < 2 || S.nstr == 0) continue;
        if (S.ny == 0) return 0;
        m = std::max(m, S.ny);
    }
    return m;
}

// bytes of one alpha-major (*na) and one beta-major (*nb) layout copy of a
// dtype's workspace; one-block spaces (and GAS spaces with owner tables) add
// one zero row after the copy (rows the owner-computes sigma_3 and the
// pair-product kernels read in place of missing ones)
void workspace_copy_sizes(const cisigma_ctx *c, size_t es, size_t *na, size_t *nb) {
    int64_t zero_row = c->cas ? c->pl[0].ld[0] : 0;
    if (c->go.ks) for (int ld : c->pl[0].ld) zero_row = std::max<int64_t>(zero_row, ld);
    *na = size_t(std::max<int64_t>(c->pl[0].size + zero_row, 1)) * es;
    *nb = size_t(std::max<int64_t>(c->pl[1].size + (c->cas ? c->pl[1].ld[0] : 0), 1)) * es;
}

// device bytes of the four layout copies of one dtype's workspace (without the
// materialised same-spin rows, which take what is free)
size_t workspace_copy_bytes(const cisigma_ctx *c, size_t es) {
    size_t na = 0, nb = 0;
    workspace_copy_sizes(c, es, &na, &nb);
    return 2 * (na + nb);
}

// rows of the materialised same-spin products (one-type spins whose pair count
// has MFMA kernels), their widest row, and whether every spin qualifies
bool ys_shape(const cisigma_ctx *c, size_t *rows, size_t *cols) {
    *rows = 0;
    *cols = 0;
    bool ok = c->cas;
    for (int s = 0; s < 2; ++s)
        if (c->sp[s].nel >= 2) {
            *rows = std::max(*rows, size_t(c->sp[s].nK) * c->sp[s].npv);
            *cols = std::max(*cols, size_t(c->pl[s].ld[0]));
            ok = ok && cis::same_spin_materialisable(c->sp[s].npv);
        }
    return ok && *rows > 0;
}

int ensure_workspace(cisigma_ctx *c, int dtype) {
    auto &W = c->ws[dtype == CISIGMA_FP32 ? 1 : 0];
    if (W.ready) return CISIGMA_OK;
    size_t es = dtype == CISIGMA_FP32 ? 4 : 8;
    size_t na = 0, nb = 0;
    workspace_copy_sizes(c, es, &na, &nb);
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess && 2 * (na + nb) + (64u << 20) > fr)
        return cis_set_error(c, CISIGMA_ENOMEM, "apply: not enough device memory for the sigma workspace");
    HIP_OR_FAIL(c, hipMalloc(&W.cp, na), "apply: workspace");
    HIP_OR_FAIL(c, hipMalloc(&W.sp, na), "apply: workspace");
    HIP_OR_FAIL(c, hipMalloc(&W.ct, nb), "apply: workspace");
    HIP_OR_FAIL(c, hipMalloc(&W.st, nb), "apply: workspace");
    // padding columns of the C copies stay zero for good
    HIP_OR_FAIL(c, hipMemset(W.cp, 0, na), "apply: workspace");
    HIP_OR_FAIL(c, hipMemset(W.ct, 0, nb), "apply: workspace");
    // materialised same-spin rows for one-type spins: column chunks (multiples of 64)
    // whose slab of the gathered copy stays near 192 MiB (inside the 256 MB Infinity
    // Cache, so the ~28 reads of each row mostly hit it; measured at CAS(16,16): 4,096
    // FP32 / 2,048 FP64 columns cut a same-spin pass 9.3 -> 8.9 ms, 19.0 -> 17.7 ms)
    // where the gathered copy is below 2 GB, and at most what fits in half of what
    // is free
    size_t rows = 0, cols = 0;
    if (ys_shape(c, &rows, &cols) && hipMemGetInfo(&fr, &tot) == hipSuccess) {
        size_t budget = fr / 2;
        size_t chunk = std::min(cols, budget / (rows * es) / cis::kTileCols * cis::kTileCols);
        const size_t xrows = size_t(std::max(c->sp[0].nstr, c->sp[1].nstr)) + 1;
        if (xrows * cols * es < (size_t(1) << 31)) {
            const size_t slab = std::max<size_t>(cis::kTileCols, (size_t(192) << 20) / (xrows * es) / cis::kTileCols *
                                                                   cis::kTileCols);
            chunk = std::min(chunk, slab);
        }
        if (chunk >= size_t(cis::kTileCols) && hipMalloc(&W.ys, rows * chunk * es) == hipSuccess)
            W.ys_chunk = int(chunk);
        else
            W.ys = nullptr;
    }
    // several types: all rows at once when they fit in half of what is free
    const int64_t ny = ys_rows_elems(c);
    if (ny > 0 && hipMemGetInfo(&fr, &tot) == hipSuccess) {
        if (size_t(ny) * es <= fr / 2 && hipMalloc(&W.ys, size_t(ny) * es) == hipSuccess)
            W.ys_chunk = 0;
        else
            W.ys = nullptr;
    }
    if (!c->side) {
        HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "apply: side stream");
        HIP_OR_FAIL(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "apply: side stream");
        HIP_OR_FAIL(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "apply: side stream");
    }
    HIP_OR_FAIL(c, hipDeviceSynchronize(), "apply: workspace");
    W.ready = true;
    return CISIGMA_OK;
}

}  // namespace

namespace cis {

namespace {

// the passes of one sigma on workspace W; own = W belongs to the context (then
// profiling events and the side stream of the overlap option may be used)
int apply_sigma_ws(cisigma_ctx *c, const void *C, void *sigma, int dtype, hipStream_t s, const Workspace &W,
                   bool own) {
    // one-type spins with room for the materialised same-spin rows avoid global atomics there
    const bool mat = c->ab_mode != 1 && W.ys != nullptr;   // W.ys only where the form applies
    if (c->deterministic && !mat)
        return cis_set_error(c, CISIGMA_EUNSUPPORTED,
                             "apply: deterministic mode: the same-spin parts of this space would need the "
                             "float-atomic kernel (no stored pair-product rows for it)");
    hipEvent_t ev[CISIGMA_NPASS + 1];
    const bool prof = own && c->profile;
    if (prof) {
        for (auto &e : ev) HIP_OR_FAIL(c, hipEventCreate(&e), "apply: profiling events");
        HIP_OR_FAIL(c, hipEventRecord(ev[0], s), "apply: profiling events");
    }
    auto mark = [&](int pass) -> hipError_t { return prof ? hipEventRecord(ev[pass + 1], s) : hipSuccess; };
    c->last_path[dtype == CISIGMA_FP32] = mat ? CISIGMA_PATH_SS_MATERIALISED : 0;
    for (int &v : c->last_shape[dtype == CISIGMA_FP32]) v = 0;
    // M_S = 0 sector (Sec. 3.3): for C(Ib, Ia) = p C(Ia, Ib) the beta-beta part
    // is p times the transposed alpha-alpha part.  The alpha-alpha part then goes
    // to the second accumulator (same shape when nalpha = nbeta), the alpha-beta
    // part alone to the first, and the output gather forms sp + st + p st^T.
    const int par = c->spin_parity;
    HIP_OR_FAIL(c, launch_scatter_in(c, C, W.cp, par ? nullptr : W.ct, dtype, s), "apply: layout conversion");
    HIP_OR_FAIL(c, mark(CISIGMA_PASS_LAYOUT_IN), "apply: profiling events");
    if (par) {
        HIP_OR_FAIL(c, launch_fill(W.sp, c->pl[0].size, dtype, s), "apply: fill");
        if (!(mat && c->sp[0].nel >= 2)) HIP_OR_FAIL(c, launch_fill(W.st, c->pl[0].size, dtype, s), "apply: fill");
    } else {
        for (int spin = 0; spin < 2; ++spin) {
            if (mat && c->sp[spin].nel >= 2) continue;   // overwritten by the gather
            HIP_OR_FAIL(c, launch_fill(spin == 0 ? W.sp : W.st, c->pl[spin].size, dtype, s), "apply: fill");
        }
    }
    HIP_OR_FAIL(c, mark(CISIGMA_PASS_CLEAR), "apply: profiling events");
    const int chunk = c->ss_chunk > 0 ? std::min(c->ss_chunk, W.ys_chunk) : W.ys_chunk;
    HIP_OR_FAIL(c, launch_sigma_same_spin(c, 0, W.cp, par ? W.st : W.sp, dtype, s, mat ? W.ys : nullptr, chunk),
                "apply: sigma_2 (alpha-alpha)");
    HIP_OR_FAIL(c, mark(CISIGMA_PASS_SIGMA_AA), "apply: profiling events");
    // the beta-beta pass (memory-bound) overlaps the alpha-beta pass (matrix-core
    // bound) on the side stream: they read different copies of C and write
    // different accumulators; it reuses the materialised rows only after the
    // alpha-alpha pass, which precedes the fork.  The events of the alpha-beta
    // pass then time it while the other runs; the beta-beta "pass" time is the
    // wait for it after that.
    const bool fork = own && !par && c->overlap && c->side;
    if (fork) {
        HIP_OR_FAIL(c, hipEventRecord(c->ev_fork, s), "apply: fork");
        HIP_OR_FAIL(c, hipStreamWaitEvent(c->side, c->ev_fork, 0), "apply: fork");
        HIP_OR_FAIL(c, launch_sigma_same_spin(c, 1, W.ct, W.st, dtype, c->side, mat ? W.ys : nullptr, chunk),
                    "apply: sigma_1 (beta-beta)");
        HIP_OR_FAIL(c, hipEventRecord(c->ev_join, c->side), "apply: join");
    }
    {
        const hipError_t e = launch_sigma_ab(c, W.cp, W.sp, dtype, s);
        if (e == hipErrorNotSupported && c->deterministic)
            return cis_set_error(c, CISIGMA_EUNSUPPORTED,
                                 "apply: deterministic mode: sigma_3 of this space would need the float-atomic "
                                 "general kernel (no owner-computes kernel covers it)");
        HIP_OR_FAIL(c, e, "apply: sigma_3 (alpha-beta)");
    }
    HIP_OR_FAIL(c, mark(CISIGMA_PASS_SIGMA_AB), "apply: profiling events");
    if (fork)
        HIP_OR_FAIL(c, hipStreamWaitEvent(s, c->ev_join, 0), "apply: join");
    else if (!par)
        HIP_OR_FAIL(c, launch_sigma_same_spin(c, 1, W.ct, W.st, dtype, s, mat ? W.ys : nullptr, chunk),
                    "apply: sigma_1 (beta-beta)");
    HIP_OR_FAIL(c, mark(CISIGMA_PASS_SIGMA_BB), "apply: profiling events");
    if (par)
        HIP_OR_FAIL(c, launch_gather_parity(c, W.sp, W.st, sigma, par, dtype, s), "apply: layout conversion");
    else
        HIP_OR_FAIL(c, launch_gather_out(c, W.sp, W.st, sigma, dtype, s), "apply: layout conversion");
    HIP_OR_FAIL(c, mark(CISIGMA_PASS_LAYOUT_OUT), "apply: profiling events");
    if (prof) {
        for (auto e : ev) c->prof_events.push_back(e);
        c->prof_pending.push_back(1);
    }
    return CISIGMA_OK;
}

}  // namespace

int apply_sigma(cisigma_ctx *c, const void *C, void *sigma, int dtype, hipStream_t s) {
    int rc = ensure_workspace(c, dtype);
    if (rc) return rc;
    return apply_sigma_ws(c, C, sigma, dtype, s, c->ws[dtype == CISIGMA_FP32 ? 1 : 0], true);
}

// The workspace in the static scratch array, laid out as the allocated one:
// alpha-major copy, its accumulator, beta-major copy, its accumulator (each
// 256-byte aligned), then as many columns of the materialised same-spin rows as
// fit (none: the same-spin parts take the atomic kernels).  Every call clears
// the two copies (padding columns and zero rows must read as zeros; another
// call may have left other data there) with fill kernels, no memset.
int apply_sigma_noalloc(cisigma_ctx *c, const void *C, void *sigma, int dtype, hipStream_t s) {
    if (!c->scratch) return cis_set_error(c, CISIGMA_EDEVICE, "apply_noalloc: scratch address not available");
    const size_t es = dtype == CISIGMA_FP32 ? 4 : 8;
    size_t na = 0, nb = 0;
    workspace_copy_sizes(c, es, &na, &nb);
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t copies = 2 * up(na) + 2 * up(nb);
    if (copies > kNoallocScratchBytes)
        return cis_set_error(c, CISIGMA_EUNSUPPORTED,
                             "apply_noalloc: the space needs " + std::to_string(copies) +
                                 " bytes of workspace, more than the " + std::to_string(kNoallocScratchBytes) +
                                 "-byte static scratch");
    unsigned char *base = static_cast<unsigned char *>(c->scratch);
    Workspace W{};
    W.cp = base;
    W.sp = base + up(na);
    W.ct = base + 2 * up(na);
    W.st = base + 2 * up(na) + up(nb);
    size_t rows = 0, cols = 0;
    if (ys_shape(c, &rows, &cols)) {
        const size_t chunk =
            std::min(cols, (kNoallocScratchBytes - copies) / (rows * es) / cis::kTileCols * cis::kTileCols);
        if (chunk >= size_t(cis::kTileCols)) {
            W.ys = base + copies;
            W.ys_chunk = int(chunk);
        }
    }
    const int64_t ny = ys_rows_elems(c);
    if (ny > 0 && size_t(ny) * es <= kNoallocScratchBytes - copies) W.ys = base + copies;
    W.ready = true;
    HIP_OR_FAIL(c, launch_fill(W.cp, int64_t(na / es), dtype, s), "apply_noalloc: clear");
    HIP_OR_FAIL(c, launch_fill(W.ct, int64_t(nb / es), dtype, s), "apply_noalloc: clear");
    return apply_sigma_ws(c, C, sigma, dtype, s, W, false);
}

int gas_set_unit_order(cisigma_ctx *c, int d, int order) {
    GasOwner &G = c->go;
    const auto &U = G.units[d];
    if (U.empty()) return CISIGMA_OK;
    const auto &A = c->sp[0];
    const size_t nu = U.size();
    std::vector<size_t> ord(nu);
    for (size_t k = 0; k < nu; ++k) ord[k] = k;
    auto work = [&](size_t k) { return double(U[k].nact) * A.tcount[U[k].ta]; };
    // The paper's batch weights (Sec. 3.1) with a unit as the batch and its allowed
    // (alpha type, beta type) blocks, restricted to the unit's columns, as the
    // batch's blocks: l_j the determinants of block j in the unit, c_j its
    // connections -- the allowed blocks (ta', tb') with ta' and tb' one excitation
    // away from its types (GAS occupations that differ by at most one electron
    // moved between spaces) -- a = sum_j c_j l_j (Eq. 10), b = (sum_j c_j) N_blocks
    // (Eq. 11).
    std::vector<double> wa(nu, 0.0), wb(nu, 0.0);
    if (order == 4 || order == 5) {
        const auto &B = c->sp[1];
        const int nta = A.ntype, ntb = B.ntype, ng = c->gas.ngas;
        auto near = [&](const std::vector<int> &occ, int t, int u) {
            int dist = 0;
            for (int g = 0; g < ng; ++g) dist += std::abs(occ[size_t(t) * ng + g] - occ[size_t(u) * ng + g]);
            return dist <= 2;
        };
        auto allowed = [&](int ta, int tb) { return c->lay.boff[size_t(ta) * ntb + tb] >= 0; };
        std::vector<double> conn(size_t(nta) * ntb, 0.0);
        for (int ta = 0; ta < nta; ++ta)
            for (int tb = 0; tb < ntb; ++tb) {
                if (!allowed(ta, tb)) continue;
                int cnt = 0;
                for (int ua = 0; ua < nta; ++ua)
                    for (int ub = 0; ub < ntb; ++ub)
                        if (allowed(ua, ub) && near(A.tocc, ta, ua) && near(B.tocc, tb, ub)) ++cnt;
                conn[size_t(ta) * ntb + tb] = cnt;
            }
        for (size_t k = 0; k < nu; ++k) {
            const int ta = U[k].ta;
            int col = 0, nblocks = 0;   // compact columns of ta: its allowed blocks in beta-type order
            double sum_cl = 0, sum_c = 0;
            for (int tb = 0; tb < ntb; ++tb) {
                if (!allowed(ta, tb)) continue;
                const int x0 = std::max(col, U[k].lo), x1 = std::min(col + B.tcount[tb], U[k].hi);
                col += B.tcount[tb];
                if (x1 <= x0) continue;
                const double cj = conn[size_t(ta) * ntb + tb];
                sum_cl += cj * double(A.tcount[ta]) * double(x1 - x0);
                sum_c += cj;
                ++nblocks;
            }
            wa[k] = sum_cl;
            wb[k] = sum_c * nblocks;
        }
    }
    if (order == 1) {
        std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
            return U[x].ta != U[y].ta ? U[x].ta < U[y].ta : U[x].lo < U[y].lo;
        });
    } else if (order == 2 || order == 3) {
        std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return work(x) > work(y); });
        if (order == 3) {
            std::vector<size_t> alt;
            for (size_t i = 0, j = nu; i < j;) {
                alt.push_back(ord[i++]);
                if (i < j) alt.push_back(ord[--j]);
            }
            ord.swap(alt);
        }
    } else if (order == 4 || order == 5) {
        const auto &w = order == 4 ? wa : wb;
        std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return w[x] > w[y]; });
    }
    std::vector<int> utab;
    int nblk = 0;
    G.launch[d].clear();
    for (size_t k : ord) {
        const auto &un = U[k];
        utab.insert(utab.end(), {un.ta, un.lo, un.hi, un.act0, un.nact, A.tstart[un.ta], nblk, 0});
        G.launch[d].push_back({nblk, A.tcount[un.ta]});
        nblk += A.tcount[un.ta];
    }
    HIP_OR_FAIL(c, hipDeviceSynchronize(), "unit order");
    drop_graphs(c);
    HIP_OR_FAIL(c, hipMemcpy(G.d_units[d], utab.data(), utab.size() * sizeof(int), hipMemcpyHostToDevice),
                "unit order");
    c->unit_order[d] = order;
    return CISIGMA_OK;
}

// Drops the owner-computes unit tables and builds them again (after a change of
// the unit width or of the one-block request), keeping each precision's unit order.
int rebuild_gas_owner(cisigma_ctx *c) {
    HIP_OR_FAIL(c, hipDeviceSynchronize(), "owner units");
    drop_graphs(c);
    GasOwner &G = c->go;
    (void)hipFree(G.d_slot); (void)hipFree(G.d_coff); (void)hipFree(G.d_g32); (void)hipFree(G.d_g64);
    for (int d = 0; d < 2; ++d) {
        (void)hipFree(G.d_act[d]);
        (void)hipFree(G.d_units[d]);
        (void)hipFree(G.plan[d].d_entries[0]);
        (void)hipFree(G.plan[d].d_entries[1]);
    }
    G = GasOwner{};
    int rc = build_gas_owner(c, c->ab_mode == 2);
    for (int d = 0; d < 2 && rc == CISIGMA_OK; ++d)
        if (c->unit_order[d]) rc = gas_set_unit_order(c, d, c->unit_order[d]);
    return rc;
}

bool workspace_fits(cisigma_ctx *c, int dtype) {
    if (c->ws[dtype == CISIGMA_FP32 ? 1 : 0].ready) return true;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return true;
    const size_t need = workspace_copy_bytes(c, dtype == CISIGMA_FP32 ? 4 : 8);
    return need + need / 8 + (256u << 20) <= fr;
}

int release_workspace(cisigma_ctx *c, int dtype) {
    auto &W = c->ws[dtype == CISIGMA_FP32 ? 1 : 0];
    if (!W.ready) return CISIGMA_OK;
    HIP_OR_FAIL(c, hipDeviceSynchronize(), "release workspace");
    drop_graphs(c);   // captured graphs name these buffers
    (void)hipFree(W.cp); (void)hipFree(W.sp); (void)hipFree(W.ct); (void)hipFree(W.st); (void)hipFree(W.ys);
    W = Workspace{};
    return CISIGMA_OK;
}

void drop_graphs(cisigma_ctx *c) {
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

int apply_sigma_graph(cisigma_ctx *c, const void *C, void *sigma, int dtype, hipStream_t s) {
    for (auto &g : c->graphs)
        if (g.C == C && g.sigma == sigma && g.dtype == dtype && g.stream == s) {
            HIP_OR_FAIL(c, hipGraphLaunch(g.exec, s), "apply: graph launch");
            c->last_path[dtype == CISIGMA_FP32] = g.path;
            return CISIGMA_OK;
        }
    // first call with these arguments: run eagerly (this call's result; it also
    // allocates the workspace and sets every kernel attribute), then capture the
    // same launches for the next calls
    int rc = apply_sigma(c, C, sigma, dtype, s);
    if (rc) return rc;
    const int path = c->last_path[dtype == CISIGMA_FP32];
    HIP_OR_FAIL(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "apply: graph capture");
    rc = apply_sigma(c, C, sigma, dtype, s);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        if (rc) return rc;
        return hip_fail(c, e != hipSuccess ? e : hipErrorUnknown, "apply: graph capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIP_OR_FAIL(c, e, "apply: graph instantiation");
    if (c->graphs.size() >= 16) {
        (void)hipGraphExecDestroy(c->graphs.front().exec);
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.push_back({C, sigma, dtype, s, exec, path});
    return CISIGMA_OK;
}

}  // namespace cis

static void prof_reset(cisigma_ctx *c) {
    for (auto e : c->prof_events) (void)hipEventDestroy(e);
    c->prof_events.clear();
    c->prof_pending.clear();
    for (double &v : c->prof_ms) v = 0;
    c->prof_calls = 0;
}

CIS_API int cisigma_pass_times(cisigma_ctx *ctx, double *ms, int *ncalls) {
    if (!ctx || !ms || !ncalls) return CISIGMA_EINVAL;
    if (!ctx->profile) return cis_set_error(ctx, CISIGMA_EINVAL, "pass_times: profiling is off");
    const size_t per = CISIGMA_NPASS + 1;
    for (size_t k = 0; k < ctx->prof_pending.size(); ++k) {
        hipEvent_t *ev = &ctx->prof_events[k * per];
        HIP_OR_FAIL(ctx, hipEventSynchronize(ev[per - 1]), "pass_times");
        for (int p = 0; p < CISIGMA_NPASS; ++p) {
            float t = 0;
            HIP_OR_FAIL(ctx, hipEventElapsedTime(&t, ev[p], ev[p + 1]), "pass_times");
            ctx->prof_ms[p] += t;
        }
        ctx->prof_calls += 1;
    }
    for (auto e : ctx->prof_events) (void)hipEventDestroy(e);
    ctx->prof_events.clear();
    ctx->prof_pending.clear();
    for (int p = 0; p < CISIGMA_NPASS; ++p) ms[p] = ctx->prof_ms[p];
    *ncalls = ctx->prof_calls;
    return CISIGMA_OK;
}

CIS_API int cisigma_last_path(const cisigma_ctx *ctx, int dtype, int *flags) {
    if (!ctx || !flags || (dtype != CISIGMA_FP32 && dtype != CISIGMA_FP64)) return CISIGMA_EINVAL;
    *flags = ctx->last_path[dtype == CISIGMA_FP32];
    return CISIGMA_OK;
}

CIS_API int cisigma_last_shape(const cisigma_ctx *ctx, int dtype, int *shape) {
    if (!ctx || !shape || (dtype != CISIGMA_FP32 && dtype != CISIGMA_FP64)) return CISIGMA_EINVAL;
    for (int i = 0; i < 4; ++i) shape[i] = ctx->last_shape[dtype == CISIGMA_FP32][i];
    return CISIGMA_OK;
}

CIS_API const char *cisigma_strerror(int status) { return status_text(status); }

CIS_API const char *cisigma_last_error(const cisigma_ctx *ctx) {
    if (!ctx) return "NULL context";
    return ctx->err.c_str();
}

CIS_API void cisigma_free(cisigma_ctx *ctx) { free_ctx(ctx); }

CIS_API int64_t cisigma_ndet(const cisigma_ctx *ctx) { return ctx ? ctx->lay.ndet : -1; }

CIS_API int cisigma_init(cisigma_ctx **out, int norb, int nalpha, int nbeta, const cisigma_gas *gas,
                         const double *h1e, const double *eri) {
    return cisigma_init_sym(out, norb, nalpha, nbeta, gas, nullptr, 0, h1e, eri);
}

CIS_API int cisigma_init_sym(cisigma_ctx **out, int norb, int nalpha, int nbeta, const cisigma_gas *gas,
                             const int *orbsym, int target, const double *h1e, const double *eri) {
    if (!out) return CISIGMA_EINVAL;
    *out = nullptr;
    if (norb < 1 || norb > 32 || nalpha < 0 || nbeta < 0 || nalpha > norb || nbeta > norb || !h1e || !eri)
        return CISIGMA_EINVAL;
    if (orbsym) {
        if (target < 0 || target > 7) return CISIGMA_EINVAL;
        for (int p = 0; p < norb; ++p)
            if (orbsym[p] < 0 || orbsym[p] > 7) return CISIGMA_EINVAL;
    }
    cisigma_ctx *c = new (std::nothrow) cisigma_ctx();
    if (!c) return CISIGMA_ENOMEM;
    c->n = norb; c->na = nalpha; c->nb = nbeta;
    c->sym = orbsym != nullptr;
    c->target = orbsym ? target : 0;
    for (int p = 0; p < norb; ++p) c->orbsym[p] = orbsym ? orbsym[p] : 0;
    // GAS
    if (gas) {
        if (gas->ngas < 1 || gas->ngas > cis::kMaxGas || !gas->norb || !gas->min_cum || !gas->max_cum) {
            free_ctx(c);
            return CISIGMA_EINVAL;
        }
        int tot = 0;
        for (int g = 0; g < gas->ngas; ++g) {
            if (gas->norb[g] < 0) { free_ctx(c); return CISIGMA_EINVAL; }
            tot += gas->norb[g];
            c->gas_norb.push_back(gas->norb[g]);
            c->gas_min.push_back(gas->min_cum[g]);
            c->gas_max.push_back(gas->max_cum[g]);
        }
        if (tot != norb) { free_ctx(c); return CISIGMA_EINVAL; }
    } else {
        c->gas_norb = {norb};
        c->gas_min = {nalpha + nbeta};
        c->gas_max = {nalpha + nbeta};
    }
    const int G = int(c->gas_norb.size());
    c->gas.n = norb;
    c->gas.ngas = G;
    {
        int first = 0;
        for (int g = 0; g < G; ++g) {
            c->gas.first[g] = first;
            uint32_t m = 0;
            for (int k = 0; k < c->gas_norb[g]; ++k) m |= 1u << (first + k);
            c->gas.mask[g] = m;
            first += c->gas_norb[g];
        }
        uint64_t mul = 1;
        for (int g = G - 1; g >= 0; --g) {
            c->gas.keymul[g] = mul;
            mul *= uint64_t(c->gas_norb[g] + 1);
        }
    }
    // integrals: finite and symmetric
    const size_t n2 = size_t(norb) * norb;
    c->h.assign(h1e, h1e + n2);
    c->g.assign(eri, eri + n2 * n2);
    double hmax = 0, gmax = 0;
    for (double v : c->h) { if (!std::isfinite(v)) { free_ctx(c); return CISIGMA_EINVAL; } hmax = std::max(hmax, std::fabs(v)); }
    for (double v : c->g) { if (!std::isfinite(v)) { free_ctx(c); return CISIGMA_EINVAL; } gmax = std::max(gmax, std::fabs(v)); }
    const double th = 1e-12 * std::max(hmax, 1.0), tg = 1e-12 * std::max(gmax, 1.0);
    for (int p = 0; p < norb; ++p)
        for (int q = 0; q < norb; ++q)
            if (std::fabs(c->h[size_t(p) * norb + q] - c->h[size_t(q) * norb + p]) > th) {
                cis_set_error(c, CISIGMA_EINVAL, "init: h1e is not symmetric");
                free_ctx(c);
                return CISIGMA_EINVAL;
            }
    auto G4 = [&](int p, int q, int r, int s) { return c->g[((size_t(p) * norb + q) * norb + r) * norb + s]; };
    for (int p = 0; p < norb; ++p)
        for (int q = 0; q < norb; ++q)
            for (int r = 0; r < norb; ++r)
                for (int s = 0; s < norb; ++s) {
                    double v = G4(p, q, r, s);
                    if (std::fabs(v - G4(q, p, r, s)) > tg || std::fabs(v - G4(p, q, s, r)) > tg ||
                        std::fabs(v - G4(r, s, p, q)) > tg) {
                        free_ctx(c);
                        return CISIGMA_EINVAL;
                    }
                }
    // with spatial symmetry the integrals must respect it: h_pq = 0 unless p and q
    // share an irrep, (pq|rs) = 0 unless the four irreps multiply to the totally
    // symmetric one (otherwise H couples the space to determinants outside it)
    if (c->sym) {
        for (int p = 0; p < norb; ++p)
            for (int q = 0; q < norb; ++q)
                if (c->orbsym[p] != c->orbsym[q] && std::fabs(c->h[size_t(p) * norb + q]) > th) {
                    cis_set_error(c, CISIGMA_EINVAL, "init: h1e breaks the orbital symmetry");
                    free_ctx(c);
                    return CISIGMA_EINVAL;
                }
        for (int p = 0; p < norb; ++p)
            for (int q = 0; q < norb; ++q)
                for (int r = 0; r < norb; ++r)
                    for (int t = 0; t < norb; ++t)
                        if ((c->orbsym[p] ^ c->orbsym[q] ^ c->orbsym[r] ^ c->orbsym[t]) != 0 &&
                            std::fabs(G4(p, q, r, t)) > tg) {
                            cis_set_error(c, CISIGMA_EINVAL, "init: eri breaks the orbital symmetry");
                            free_ctx(c);
                            return CISIGMA_EINVAL;
                        }
    }
    // GAS occupation tuples per spin, kept when they pair with a tuple of the other spin
    std::vector<std::vector<int>> tup[2];
    for (int s = 0; s < 2; ++s) {
        std::vector<int> cur(G, 0);
        enum_tuples(c->gas_norb, s == 0 ? nalpha : nbeta, 0, cur, tup[s]);
        std::sort(tup[s].begin(), tup[s].end());
    }
    std::vector<char> keep[2] = {std::vector<char>(tup[0].size(), 0), std::vector<char>(tup[1].size(), 0)};
    for (size_t a = 0; a < tup[0].size(); ++a)
        for (size_t b = 0; b < tup[1].size(); ++b)
            if (pair_allowed(c, tup[0][a].data(), tup[1][b].data())) keep[0][a] = keep[1][b] = 1;
    for (int s = 0; s < 2; ++s) {
        auto &T = c->sp[s];
        T.nel = s == 0 ? nalpha : nbeta;
        T.graw.assign(1, 0);
        for (size_t i = 0; i < tup[s].size(); ++i) {
            if (!keep[s][i]) continue;
            uint64_t cnt = 1, key = 0;
            for (int g = 0; g < G; ++g) {
                cnt *= binom(c->gas_norb[g], tup[s][i][g]);
                key += uint64_t(tup[s][i][g]) * c->gas.keymul[g];
            }
            if (uint64_t(T.graw.back()) + cnt > (uint64_t(1) << (c->sym ? 27 : 21)) - 1) {
                cis_set_error(c, CISIGMA_EUNSUPPORTED, "init: too many strings of one spin");
                free_ctx(c);
                return CISIGMA_EUNSUPPORTED;
            }
            for (int g = 0; g < G; ++g) T.gtocc.push_back(tup[s][i][g]);
            T.gkey.push_back(key);
            T.graw.push_back(T.graw.back() + int(cnt));
        }
        T.ngtype = int(T.gkey.size());
    }
    if (!c->sym) {
        // the types are the GAS types; string index = raw index
        for (int s = 0; s < 2; ++s) {
            auto &T = c->sp[s];
            T.tocc = T.gtocc;
            T.tstart = T.graw;
            T.tcount.clear();
            for (int t = 0; t < T.ngtype; ++t) T.tcount.push_back(T.graw[t + 1] - T.graw[t]);
            T.tirrep.assign(T.ngtype, 0);
            T.ntype = T.ngtype;
            T.nstr = T.tstart.back();
        }
    } else {
        // spatial symmetry: irrep of every raw string (the strings of a GAS type in
        // ascending order: mixed radix over the GAS spaces, space 0 fastest)
        std::vector<std::vector<uint8_t>> irr(2);
        std::vector<std::vector<int>> cnt(2);           // [gtype * 8 + irrep]
        for (int s = 0; s < 2; ++s) {
            auto &T = c->sp[s];
            irr[s].resize(size_t(T.graw.back()));
            cnt[s].assign(size_t(T.ngtype) * 8, 0);
            for (int gt = 0; gt < T.ngtype; ++gt) {
                std::vector<std::vector<int>> sub(G);   // irreps of the sub-strings of each space
                for (int g = 0; g < G; ++g) {
                    const int m = c->gas_norb[g], k = T.gtocc[size_t(gt) * G + g];
                    uint64_t x = (uint64_t(1) << k) - 1;
                    for (uint64_t q = 0; q < binom(m, k); ++q) {
                        int ir = 0;
                        for (int p = 0; p < m; ++p)
                            if ((x >> p) & 1u) ir ^= c->orbsym[c->gas.first[g] + p];
                        sub[g].push_back(ir);
                        if (x == 0) break;
                        const uint64_t lo = x & (~x + 1), r = x + lo;
                        x = (((r ^ x) >> 2) / lo) | r;
                    }
                }
                for (int raw = T.graw[gt]; raw < T.graw[gt + 1]; ++raw) {
                    uint32_t rem = uint32_t(raw - T.graw[gt]);
                    int ir = 0;
                    for (int g = 0; g < G; ++g) {
                        const uint32_t base = uint32_t(sub[g].size());
                        ir ^= sub[g][rem % base];
                        rem /= base;
                    }
                    irr[s][size_t(raw)] = uint8_t(ir);
                    ++cnt[s][size_t(gt) * 8 + ir];
                }
            }
        }
        // types (GAS type, irrep) with strings, kept when they pair with a type of the
        // other spin: GAS bounds and irreps multiplying to the target
        std::vector<char> tkeep[2] = {std::vector<char>(size_t(c->sp[0].ngtype) * 8, 0),
                                      std::vector<char>(size_t(c->sp[1].ngtype) * 8, 0)};
        for (int a = 0; a < c->sp[0].ngtype; ++a)
            for (int b = 0; b < c->sp[1].ngtype; ++b) {
                if (!pair_allowed(c, &c->sp[0].gtocc[size_t(a) * G], &c->sp[1].gtocc[size_t(b) * G])) continue;
                for (int ia = 0; ia < 8; ++ia) {
                    const int ib = ia ^ c->target;
                    if (cnt[0][size_t(a) * 8 + ia] > 0 && cnt[1][size_t(b) * 8 + ib] > 0)
                        tkeep[0][size_t(a) * 8 + ia] = tkeep[1][size_t(b) * 8 + ib] = 1;
                }
            }
        for (int s = 0; s < 2; ++s) {
            auto &T = c->sp[s];
            T.tstart.assign(1, 0);
            std::vector<int> tid(size_t(T.ngtype) * 8, -1);
            for (int gt = 0; gt < T.ngtype; ++gt)
                for (int ir = 0; ir < 8; ++ir) {
                    if (!tkeep[s][size_t(gt) * 8 + ir]) continue;
                    tid[size_t(gt) * 8 + ir] = int(T.tcount.size());
                    for (int g = 0; g < G; ++g) T.tocc.push_back(T.gtocc[size_t(gt) * G + g]);
                    T.tirrep.push_back(ir);
                    T.tcount.push_back(cnt[s][size_t(gt) * 8 + ir]);
                    T.tstart.push_back(T.tstart.back() + T.tcount.back());
                }
            T.ntype = int(T.tcount.size());
            T.nstr = T.tstart.back();
            if (T.nstr > (1 << 21) - 1) {
                cis_set_error(c, CISIGMA_EUNSUPPORTED, "init: more than 2^21-1 strings of one spin");
                free_ctx(c);
                return CISIGMA_EUNSUPPORTED;
            }
            // raw -> string index: strings of a type in ascending raw (= bitmask) order
            T.remap.assign(size_t(T.graw.back()), -1);
            std::vector<int> fill(T.tstart.begin(), T.tstart.end() - 1);
            for (int gt = 0; gt < T.ngtype; ++gt)
                for (int raw = T.graw[gt]; raw < T.graw[gt + 1]; ++raw) {
                    const int t = tid[size_t(gt) * 8 + irr[s][size_t(raw)]];
                    if (t >= 0) T.remap[size_t(raw)] = fill[size_t(t)]++;
                }
        }
    }
    // blocks in alpha-type-major order
    {
        auto &L = c->lay;
        const auto &A = c->sp[0], &B = c->sp[1];
        L.boff.assign(size_t(A.ntype) * B.ntype, -1);
        int64_t off = 0;
        for (int a = 0; a < A.ntype; ++a)
            for (int b = 0; b < B.ntype; ++b)
                if (block_allowed(c, a, b)) {
                    L.boff[size_t(a) * B.ntype + b] = off;
                    L.blk_a.push_back(a);
                    L.blk_b.push_back(b);
                    L.blk_off.push_back(off);
                    off += int64_t(A.tcount[a]) * B.tcount[b];
                }
        L.blk_off.push_back(off);
        L.nblk = int(L.blk_a.size());
        L.ndet = off;
        if (off == 0) {
            free_ctx(c);
            return CISIGMA_EINVAL;
        }
    }
    c->cas = !c->sym && c->sp[0].ntype == 1 && c->sp[1].ntype == 1;
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    // set-up of cisigma_apply_noalloc: the device address of this device's scratch
    // array (looked up once per device, with it current)
    if (he == hipSuccess) {
        c->dev = dev;
        c->scratch = noalloc_scratch(dev, &he);
    }
    if (he != hipSuccess) {
        int rc = hip_fail(c, he, "init: device");
        free_ctx(c);
        return rc;
    }
    int rc = build_layouts(c);
    if (!rc) rc = build_integrals(c);
    if (!rc) {
        for (int s = 0; s < 2 && !rc; ++s) {
            hipError_t e = cis::build_string_tables(c, s);
            if (e != hipSuccess) rc = hip_fail(c, e, "init: string tables");
        }
    }
    if (!rc) {
        hipError_t e = cis::build_diag_tables(c);
        if (e != hipSuccess) rc = hip_fail(c, e, "init: diagonal tables");
    }
    if (!rc) rc = build_active_tiles(c);
    if (!rc) rc = build_scatter_plan(c);
    if (!rc) rc = build_gas_owner(c, false);
    if (!rc) rc = build_same_spin_rows(c);
    if (rc) {
        std::fprintf(stderr, "cisigma_init: %s\n", c->err.c_str());
        free_ctx(c);
        return rc;
    }
    *out = c;
    return CISIGMA_OK;
}

CIS_API int cisigma_layout(const cisigma_ctx *ctx, int *nblocks, int64_t *block_offset, int *alpha_type,
                           int *beta_type, int *nalpha_str, int *nbeta_str) {
    if (!ctx || !nblocks) return CISIGMA_EINVAL;
    const auto &L = ctx->lay;
    *nblocks = L.nblk;
    for (int b = 0; b < L.nblk; ++b) {
        if (block_offset) block_offset[b] = L.blk_off[b];
        if (alpha_type) alpha_type[b] = L.blk_a[b];
        if (beta_type) beta_type[b] = L.blk_b[b];
        if (nalpha_str) nalpha_str[b] = ctx->sp[0].tcount[L.blk_a[b]];
        if (nbeta_str) nbeta_str[b] = ctx->sp[1].tcount[L.blk_b[b]];
    }
    if (block_offset) block_offset[L.nblk] = L.ndet;
    return CISIGMA_OK;
}

CIS_API int cisigma_address(const cisigma_ctx *ctx, uint32_t alpha_bits, uint32_t beta_bits, int64_t *index) {
    if (!ctx || !index) return CISIGMA_EINVAL;
    *index = -1;
    int64_t a = host_string_index(ctx, 0, alpha_bits), b = host_string_index(ctx, 1, beta_bits);
    if (a < 0 || b < 0) return CISIGMA_OK;
    const auto &A = ctx->sp[0], &B = ctx->sp[1];
    int ta = int(std::upper_bound(A.tstart.begin(), A.tstart.end(), int(a)) - A.tstart.begin()) - 1;
    int tb = int(std::upper_bound(B.tstart.begin(), B.tstart.end(), int(b)) - B.tstart.begin()) - 1;
    int64_t off = ctx->lay.boff[size_t(ta) * B.ntype + tb];
    if (off < 0) return CISIGMA_OK;
    *index = off + (a - A.tstart[ta]) * B.tcount[tb] + (b - B.tstart[tb]);
    return CISIGMA_OK;
}

CIS_API int cisigma_hmat_block(cisigma_ctx *ctx, int n, const int64_t *rows, int m, const int64_t *cols,
                               double *out) {
    if (!ctx || n < 0 || m < 0 || (n > 0 && !rows) || (m > 0 && !cols) || (n > 0 && m > 0 && !out))
        return ctx ? cis_set_error(ctx, CISIGMA_EINVAL, "hmat_block: bad arguments") : CISIGMA_EINVAL;
    std::vector<uint32_t> astr(ctx->sp[0].nstr), bstr(ctx->sp[1].nstr);
    if (!astr.empty())
        HIP_OR_FAIL(ctx, hipMemcpy(astr.data(), ctx->sp[0].d_str, astr.size() * 4, hipMemcpyDeviceToHost), "hmat_block");
    if (!bstr.empty())
        HIP_OR_FAIL(ctx, hipMemcpy(bstr.data(), ctx->sp[1].d_str, bstr.size() * 4, hipMemcpyDeviceToHost), "hmat_block");
    std::vector<uint32_t> ca(m), cb(m);
    for (int j = 0; j < m; ++j)
        if (!cis::det_strings(ctx, cols[j], astr, bstr, &ca[j], &cb[j]))
            return cis_set_error(ctx, CISIGMA_EINVAL, "hmat_block: column index out of range");
    for (int i = 0; i < n; ++i) {
        uint32_t a, b;
        if (!cis::det_strings(ctx, rows[i], astr, bstr, &a, &b))
            return cis_set_error(ctx, CISIGMA_EINVAL, "hmat_block: row index out of range");
        for (int j = 0; j < m; ++j) out[size_t(i) * m + j] = cis::hmat_element(ctx, a, b, ca[j], cb[j]);
    }
    return CISIGMA_OK;
}

namespace {
__global__ void k_fill_ramp(void *x, int64_t n, int fp32) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = 1.0 / double(1 + (i % 977));
        if (fp32) static_cast<float *>(x)[i] = float(v); else static_cast<double *>(x)[i] = v;
    }
}
}  // namespace

CIS_API int cisigma_autotune(cisigma_ctx *ctx, int dtype, int reps, char *report, int report_len) {
    if (!ctx) return CISIGMA_EINVAL;
    if ((dtype != CISIGMA_FP32 && dtype != CISIGMA_FP64) || reps < 1 || reps > 100 || (report_len > 0 && !report))
        return cis_set_error(ctx, CISIGMA_EINVAL, "autotune: bad arguments");
    const int d = dtype == CISIGMA_FP32 ? 1 : 0;
    const size_t es = dtype == CISIGMA_FP32 ? 4 : 8;
    const int64_t N = ctx->lay.ndet;
    const int parity = ctx->spin_parity;
    const int graph = ctx->graph_mode, prof = ctx->profile;
    std::string rep;
    void *C = nullptr, *S = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto done = [&](int rc) {
        (void)hipFree(C); (void)hipFree(S);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        ctx->spin_parity = parity; ctx->graph_mode = graph; ctx->profile = prof;
        if (report_len > 0) {
            const size_t n = std::min(rep.size(), size_t(report_len - 1));
            std::memcpy(report, rep.data(), n);
            report[n] = 0;
        }
        return rc;
    };
    // timed on a fixed vector, eager launches, no spin-parity restriction
    ctx->spin_parity = 0; ctx->graph_mode = 0; ctx->profile = 0;
    hipError_t e = hipMalloc(&C, size_t(std::max<int64_t>(N, 1)) * es);
    if (e == hipSuccess) e = hipMalloc(&S, size_t(std::max<int64_t>(N, 1)) * es);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return done(hip_fail(ctx, e, "autotune: buffers"));
    const hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(k_fill_ramp, dim3(1024), dim3(256), 0, s, C, N, int(d == 1));
    auto time_apply = [&](float *ms) -> int {
        int rc = cis::apply_sigma(ctx, C, S, dtype, s);    // warm-up (allocates the workspace once)
        if (rc) return rc;
        HIP_OR_FAIL(ctx, hipEventRecord(e0, s), "autotune: events");
        for (int r = 0; r < reps && rc == 0; ++r) rc = cis::apply_sigma(ctx, C, S, dtype, s);
        if (rc) return rc;
        HIP_OR_FAIL(ctx, hipEventRecord(e1, s), "autotune: events");
        HIP_OR_FAIL(ctx, hipEventSynchronize(e1), "autotune: events");
        HIP_OR_FAIL(ctx, hipEventElapsedTime(ms, e0, e1), "autotune: events");
        *ms /= float(reps);
        return CISIGMA_OK;
    };
    char line[160];
    {
        float ms = 0;
        const int rc = time_apply(&ms);
        if (rc) return done(rc);
        std::snprintf(line, sizeof line, "as set: %.3f ms per sigma\n", double(ms));
        rep += line;
    }
    // knob 0: unit width (rows cut where a piece is longer than the LDS or than this)
    if (!ctx->go.units[d].empty()) {
        const int keep = ctx->unit_cols;
        int best = keep;
        float best_ms = 0;
        const int cands[] = {0, 16384, 8192, 4096};
        for (int k = 0; k < 4; ++k) {
            ctx->unit_cols = cands[k];
            int rc = cis::rebuild_gas_owner(ctx);
            float ms = 0;
            if (rc == 0 && !ctx->go.units[d].empty()) rc = time_apply(&ms);
            else if (rc == 0) continue;          // no units at this width: not a candidate
            if (rc) { ctx->unit_cols = keep; cis::rebuild_gas_owner(ctx); return done(rc); }
            std::snprintf(line, sizeof line, "unit_cols %d%s: %.3f ms per sigma\n", cands[k],
                          cands[k] == 0 ? " (the LDS)" : "", double(ms));
            rep += line;
            if (best_ms == 0 || ms < best_ms) { best = cands[k]; best_ms = ms; }
        }
        ctx->unit_cols = best;
        const int rc = cis::rebuild_gas_owner(ctx);
        if (rc) return done(rc);
        std::snprintf(line, sizeof line, "unit_cols -> %d\n", best);
        rep += line;
    }
    // knob 1: launch order of the GAS owner units of this precision
    if (!ctx->go.units[d].empty()) {
        int best = ctx->unit_order[d];
        float best_ms = 0;
        for (int order = 0; order < 6; ++order) {
            int rc = cis::gas_set_unit_order(ctx, d, order);
            float ms = 0;
            if (rc == 0) rc = time_apply(&ms);
            if (rc) return done(rc);
            std::snprintf(line, sizeof line, "gas_unit_order %d: %.3f ms per sigma\n", order, double(ms));
            rep += line;
            if (order == 0 || ms < best_ms) { best = order; best_ms = ms; }
        }
        int rc = cis::gas_set_unit_order(ctx, d, best);
        if (rc) return done(rc);
        std::snprintf(line, sizeof line, "gas_unit_order -> %d\n", best);
        rep += line;
    }
    // knob 2: column split of the grid of the same-spin kernel of spaces with several
    // types (atomic or row-store form); one-block spaces with their rows stored use
    // their own kernel.  (The workspace exists now: rows are stored exactly when
    // they were allocated.)
    const bool split_used = !(ctx->cas && ctx->ab_mode != 1 && ctx->ws[d].ys != nullptr);
    if (split_used && (ctx->sp[0].nel >= 2 || ctx->sp[1].nel >= 2)) {
        int best = 0;
        float best_ms = 0;
        const int cands[] = {0, 1, 2, 4, 8, 16, 32};
        for (int k = 0; k < 7; ++k) {
            cis::drop_graphs(ctx);
            ctx->ss_split = cands[k];
            float ms = 0;
            const int rc = time_apply(&ms);
            if (rc) return done(rc);
            std::snprintf(line, sizeof line, "same_spin_split %d%s: %.3f ms per sigma\n", cands[k],
                          cands[k] == 0 ? " (heuristic)" : "", double(ms));
            rep += line;
            if (k == 0 || ms < best_ms) { best = cands[k]; best_ms = ms; }
        }
        cis::drop_graphs(ctx);
        ctx->ss_split = best;
        std::snprintf(line, sizeof line, "same_spin_split -> %d\n", best);
        rep += line;
    }
    if (rep.empty()) rep = "nothing to tune for this space and precision\n";
    return done(CISIGMA_OK);
}

CIS_API int cisigma_strings(const cisigma_ctx *ctx, int spin, uint32_t *out, int *nstr) {
    if (!ctx || !nstr || spin < 0 || spin > 1) return CISIGMA_EINVAL;
    const auto &T = ctx->sp[spin];
    *nstr = T.nstr;
    if (out && T.nstr > 0) {
        hipError_t e = hipMemcpy(out, T.d_str, size_t(T.nstr) * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(const_cast<cisigma_ctx *>(ctx), e, "strings");
    }
    return CISIGMA_OK;
}

CIS_API int cisigma_excitations(const cisigma_ctx *ctx, int spin, uint32_t *out, int *per_string, int *nstr) {
    if (!ctx || !per_string || !nstr || spin < 0 || spin > 1) return CISIGMA_EINVAL;
    const auto &T = ctx->sp[spin];
    *nstr = T.nstr;
    *per_string = T.nexc;
    if (out && T.nstr > 0 && T.nexc > 0) {
        hipError_t e = hipMemcpy(out, T.d_exc, size_t(T.nstr) * T.nexc * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(const_cast<cisigma_ctx *>(ctx), e, "excitations");
    }
    return CISIGMA_OK;
}

CIS_API int cisigma_set_option(cisigma_ctx *ctx, int key, double value) {
    if (!ctx) return CISIGMA_EINVAL;
    if (!std::isfinite(value)) return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: value is not finite");
    switch (key) {
        case CISIGMA_OPT_PRECISION:
            if (value != CISIGMA_FP64 && value != CISIGMA_FP32)
                return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: precision must be FP64 or FP32");
            ctx->precision = int(value);
            return CISIGMA_OK;
        case CISIGMA_OPT_MAX_SPACE:
            if (value < 2 || value > 512) return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: max_space out of range");
            ctx->max_space = int(value);
            return CISIGMA_OK;
        case CISIGMA_OPT_MAX_ITER:
            if (value < 1 || value > 100000) return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: max_iter out of range");
            ctx->max_iter = int(value);
            return CISIGMA_OK;
        case CISIGMA_OPT_REFINE_EVERY:
            if (value < 0 || value > 100000) return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: refine_every out of range");
            ctx->refine_every = int(value);
            return CISIGMA_OK;
        case CISIGMA_OPT_RESID_TOL:
            if (value <= 0) return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: resid_tol must be positive");
            ctx->resid_tol = value;
            return CISIGMA_OK;
        case CISIGMA_OPT_VERBOSE:
            ctx->verbose = int(value);
            return CISIGMA_OK;
        case CISIGMA_OPT_SIGMA_PATH: {
            cis::drop_graphs(ctx);
            if (value < 0 || value > 3)
                return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: sigma path must be 0, 1, 2 or 3");
            const bool rebuild = ctx->cas && (value == 2) != (ctx->ab_mode == 2);
            ctx->ab_mode = int(value);
            return rebuild ? cis::rebuild_gas_owner(ctx) : CISIGMA_OK;
        }
        case CISIGMA_OPT_DETERMINISTIC:
            if (value != 0 && value != 1)
                return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: deterministic must be 0 or 1");
            ctx->deterministic = int(value);
            return CISIGMA_OK;
        case CISIGMA_OPT_UNIT_LAUNCH:
            if (value != 0 && value != 1) return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: unit launch must be 0 or 1");
            cis::drop_graphs(ctx);
            ctx->unit_launch = int(value);
            return CISIGMA_OK;
        case CISIGMA_OPT_UNIT_COLS:
            if (value < 0 || value > 65536 || value != std::floor(value) || (value > 0 && value < 64))
                return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: unit columns must be 0 or 64..65536");
            ctx->unit_cols = int(value);
            return cis::rebuild_gas_owner(ctx);
        case CISIGMA_OPT_SS_CHUNK:
            cis::drop_graphs(ctx);
            if (value < 0 || value > (1 << 30) || value != std::floor(value) || int64_t(value) % cis::kTileCols)
                return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: same-spin chunk must be a non-negative multiple of 64");
            ctx->ss_chunk = int(value);
            return CISIGMA_OK;
        case CISIGMA_OPT_GAS_UNIT_ORDER: {
            if (value < 0 || value > 5) return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: unit order out of range");
            int rc = cis::gas_set_unit_order(ctx, 0, int(value));
            if (rc == CISIGMA_OK) rc = cis::gas_set_unit_order(ctx, 1, int(value));
            return rc;
        }
        case CISIGMA_OPT_SS_SPLIT:
            if (value < 0 || value > 64) return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: split out of range");
            cis::drop_graphs(ctx);
            ctx->ss_split = int(value);
            return CISIGMA_OK;
        case CISIGMA_OPT_LOW_MEMORY:
            ctx->low_memory = value != 0;
            return CISIGMA_OK;
        case CISIGMA_OPT_PSPACE:
            if (value < 0 || value > 2048) return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: pspace out of range");
            ctx->pspace = int(value);
            return CISIGMA_OK;
        case CISIGMA_OPT_THICK_RESTART:
            ctx->thick_restart = value != 0;
            return CISIGMA_OK;
        case CISIGMA_OPT_OVERLAP:
            cis::drop_graphs(ctx);
            ctx->overlap = value != 0;
            return CISIGMA_OK;
        case CISIGMA_OPT_GRAPH:
            cis::drop_graphs(ctx);
            ctx->graph_mode = value != 0;
            return CISIGMA_OK;
        case CISIGMA_OPT_SPIN_PARITY:
            cis::drop_graphs(ctx);
            if (value != 0 && value != 1 && value != -1)
                return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: spin parity must be -1, 0 or +1");
            if (value != 0 && ctx->sp[0].nel != ctx->sp[1].nel)
                return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: spin parity needs nalpha = nbeta");
            if (value != 0 && !ctx->spin_sym)
                return cis_set_error(ctx, CISIGMA_EUNSUPPORTED,
                                     "set_option: spin parity needs alpha and beta tables and blocks that mirror each other");
            ctx->spin_parity = int(value);
            return CISIGMA_OK;
        case CISIGMA_OPT_PROFILE:
            prof_reset(ctx);
            ctx->profile = value != 0;
            return CISIGMA_OK;
        default:
            return cis_set_error(ctx, CISIGMA_EINVAL, "set_option: unknown key");
    }
}

CIS_API int cisigma_set_log(cisigma_ctx *ctx, const char *path) {
    if (!ctx) return CISIGMA_EINVAL;
    ctx->log_path = path ? path : "";
    return CISIGMA_OK;
}

CIS_API int cisigma_apply(cisigma_ctx *ctx, const void *C, void *sigma, int dtype, void *stream) {
    if (!ctx) return CISIGMA_EINVAL;
    if (!C || !sigma) return cis_set_error(ctx, CISIGMA_EINVAL, "apply: NULL vector");
    if (dtype != CISIGMA_FP32 && dtype != CISIGMA_FP64) return cis_set_error(ctx, CISIGMA_EINVAL, "apply: bad dtype");
    const size_t bytes = size_t(ctx->lay.ndet) * (dtype == CISIGMA_FP32 ? 4 : 8);
    const char *a = static_cast<const char *>(C), *b = static_cast<const char *>(sigma);
    if (a < b + bytes && b < a + bytes) return cis_set_error(ctx, CISIGMA_EINVAL, "apply: C and sigma overlap");
    if (ctx->graph_mode && stream && !ctx->profile)
        return cis::apply_sigma_graph(ctx, C, sigma, dtype, static_cast<hipStream_t>(stream));
    return cis::apply_sigma(ctx, C, sigma, dtype, static_cast<hipStream_t>(stream));
}

CIS_API int cisigma_apply_noalloc(cisigma_ctx *ctx, const void *C, void *sigma, int dtype, void *stream) {
    if (!ctx) return CISIGMA_EINVAL;
    if (!C || !sigma) return cis_set_error(ctx, CISIGMA_EINVAL, "apply_noalloc: NULL vector");
    if (dtype != CISIGMA_FP32 && dtype != CISIGMA_FP64)
        return cis_set_error(ctx, CISIGMA_EINVAL, "apply_noalloc: bad dtype");
    const size_t bytes = size_t(ctx->lay.ndet) * (dtype == CISIGMA_FP32 ? 4 : 8);
    const char *a = static_cast<const char *>(C), *b = static_cast<const char *>(sigma);
    if (a < b + bytes && b < a + bytes) return cis_set_error(ctx, CISIGMA_EINVAL, "apply_noalloc: C and sigma overlap");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ctx->dev)
        return cis_set_error(ctx, CISIGMA_EINVAL, "apply_noalloc: the current device is not the context's");
    return cis::apply_sigma_noalloc(ctx, C, sigma, dtype, static_cast<hipStream_t>(stream));
}

CIS_API int cisigma_rdm(cisigma_ctx *ctx, const void *C, int dtype, double *rdm1, double *rdm2, void *stream) {
    if (!ctx) return CISIGMA_EINVAL;
    if (!C || !rdm1 || !rdm2) return cis_set_error(ctx, CISIGMA_EINVAL, "rdm: NULL pointer");
    if (dtype != CISIGMA_FP32 && dtype != CISIGMA_FP64) return cis_set_error(ctx, CISIGMA_EINVAL, "rdm: bad dtype");
    if (!ctx->cas || ctx->n > 16)
        return cis_set_error(ctx, CISIGMA_EUNSUPPORTED, "rdm: built for one-block spaces of at most 16 orbitals");
    if (cis::rdm_lds_bytes(ctx, dtype) > 160 * 1024)
        return cis_set_error(ctx, CISIGMA_EUNSUPPORTED, "rdm: the alpha-major row does not fit the LDS");
    int rc = ensure_workspace(ctx, dtype);
    if (rc) return rc;
    const size_t need = cis::rdm_part_elems(ctx);
    if (ctx->rdm_elems < need) {
        (void)hipFree(ctx->d_rdm);
        ctx->d_rdm = nullptr;
        ctx->rdm_elems = 0;
        HIP_OR_FAIL(ctx, hipMalloc(&ctx->d_rdm, need * sizeof(double)), "rdm: partial-sum buffer");
        ctx->rdm_elems = need;
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    auto &W = ctx->ws[dtype == CISIGMA_FP32 ? 1 : 0];
    HIP_OR_FAIL(ctx, cis::launch_scatter_in(ctx, C, W.cp, nullptr, dtype, s), "rdm: layout conversion");
    HIP_OR_FAIL(ctx, cis::launch_rdm(ctx, W.cp, dtype, ctx->d_rdm, rdm1, rdm2, s), "rdm: density kernels");
    return CISIGMA_OK;
}

CIS_API int cisigma_hdiag(cisigma_ctx *ctx, double *hdiag, void *stream) {
    if (!ctx) return CISIGMA_EINVAL;
    if (!hdiag) return cis_set_error(ctx, CISIGMA_EINVAL, "hdiag: NULL output");
    HIP_OR_FAIL(ctx, cis::launch_hdiag(ctx, hdiag, static_cast<hipStream_t>(stream)), "hdiag");
    return CISIGMA_OK;
}

CIS_API int cisigma_davidson(cisigma_ctx *ctx, int nroots, double tol, double *energies, void *vecs,
                             cisigma_stats *stats) {
    if (!ctx) return CISIGMA_EINVAL;
    if (nroots < 1 || nroots > 64 || nroots > ctx->lay.ndet || !energies || !(tol > 0) || !std::isfinite(tol))
        return cis_set_error(ctx, CISIGMA_EINVAL, "davidson: bad nroots, tol or energies");
    return cis::davidson(ctx, nroots, tol, energies, vecs, stats);
}
