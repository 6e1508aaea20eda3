// C ABI of libsylt: argument validation, plan construction (Schur factors,
// separation, transform-pass and sweep-tile planning), and the solve drivers.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <new>

#include "sylt_internal.h"

namespace sylt {

int sweep_max_partial_block();

namespace {

constexpr int kSchurIterPerN = 30;
constexpr int64_t kTransformTileCap = 8192;  // complex entries per transform tile
constexpr int64_t kResidualTileCap = 5120;   // two tiles (X and accumulator), 160 KB
constexpr int64_t kResidualMfmaTileCap = kResidualMfmaCap;  // two tiles and the A fragments, <= 160 KB

int status_of(hipError_t e)
{
    if (e == hipSuccess) return SYLT_OK;
    if (e == hipErrorOutOfMemory) return SYLT_E_OUT_OF_MEMORY;
    return SYLT_E_DEVICE;
}

#define SYLT_TRY(expr)                          \
    do {                                        \
        hipError_t _e = (expr);                 \
        if (_e != hipSuccess) return status_of(_e); \
    } while (0)

int validate_shape(int N, const int64_t *n)
{
    if (N < 1 || !n) return SYLT_E_INVALID_ARG;
    if (N > kMaxModes) return SYLT_E_UNSUPPORTED;
    long double tot = 1;
    for (int k = 0; k < N; ++k) {
        if (n[k] < 1) return SYLT_E_INVALID_ARG;
        if (n[k] > kMaxExtent) return SYLT_E_UNSUPPORTED;
        tot *= (long double)n[k];
    }
    if (tot >= (long double)(1ull << 62)) return SYLT_E_UNSUPPORTED;
    return SYLT_OK;
}

int64_t pow2_ceil(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

int ilog2(int64_t v)
{
    int s = 0;
    while ((int64_t(1) << s) < v) ++s;
    return s;
}

void plan_pass_list(sylt_plan_s &p, int64_t cap, std::vector<PassDesc> &out)
{
    out.clear();
    const int M = p.M;
    int a = 0;
    while (a < M) {
        int64_t Lin = 1;
        for (int j = 0; j < a; ++j) Lin *= p.cdim[j];
        // inner run: 16 entries (256 B) when that still fuses as many modes as
        // 8 entries (128 B, one cache line) would; the whole low part if shorter
        auto group_end = [&](int64_t lbv) {
            int bb = a + 1;
            int64_t GG = p.cdim[a];
            while (bb < M && (int64_t)(bb - a) < kMaxGroup && lbv * GG * p.cdim[bb] <= cap)
                GG *= p.cdim[bb++];
            return bb;
        };
        int64_t lb = a == 0 ? 1 : std::min<int64_t>(16, pow2_ceil(Lin));
        if (lb == 16 && group_end(8) > group_end(16)) lb = 8;
        const int b = group_end(lb);
        int64_t G = 1;
        int maxn = 0;
        for (int j = a; j < b; ++j) {
            G *= p.cdim[j];
            maxn = std::max(maxn, p.cdim[j]);
        }
        int64_t Rout = 1;
        for (int j = b; j < M; ++j) Rout *= p.cdim[j];
        PassDesc pd{};
        pd.Lin = Lin;
        pd.G = G;
        pd.Rout = Rout;
        pd.lb = (int)lb;
        pd.lbshift = ilog2(lb);
        pd.rb = (int)std::max<int64_t>(1, std::min<int64_t>(Rout, cap / (lb * G)));
        pd.ntl = (Lin + lb - 1) / lb;
        pd.ntr = (Rout + pd.rb - 1) / pd.rb;
        pd.ng = b - a;
        int64_t gs = 1;
        pd.uniform_n = p.cdim[a];
        for (int q = 0; q < pd.ng; ++q) {
            const int j = a + q;
            pd.gd[q] = p.cdim[j];
            pd.gs[q] = (int)gs;
            gs *= p.cdim[j];
            pd.moff[q] = p.moff[p.cmode[j]];
            if (p.cdim[j] != pd.uniform_n) pd.uniform_n = 0;
        }
        pd.maxn = maxn;
        out.push_back(pd);
        a = b;
    }
}

}  // namespace

void plan_passes(sylt_plan_s &p)
{
    plan_pass_list(p, kTransformTileCap, p.passes);
    // the ping-pong (extent > 24) transform variant needs two tiles
    for (PassDesc &pd : p.passes) {
        if (pd.maxn > 24 && pd.lb * pd.G * pd.rb * 2 > kTransformTileCap) {
            std::vector<PassDesc> half;
            plan_pass_list(p, kTransformTileCap / 2, half);
            p.passes = half;
            break;
        }
    }
    plan_pass_list(p, kResidualTileCap, p.rpasses);
    // the matrix-core residual passes: smaller tiles leave room for the A
    // fragments; used when every pass has one extent of 8, 16 or 19
    plan_pass_list(p, kResidualMfmaTileCap, p.mrpasses);
    p.residual_mfma = !p.mrpasses.empty();
    for (const PassDesc &pd : p.mrpasses) {
        const int n = pd.uniform_n;
        if ((n != 8 && n != 16 && n != 19) || residual_mfma_lds(pd) > std::min<size_t>(max_lds_bytes(), 160 * 1024))
            p.residual_mfma = false;
    }
}

size_t max_lds_bytes()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 65536;
    return (size_t)v;
}

// Sweep tiling: choose the block size b_j of every compressed mode to
// minimise the modelled time of the tile wavefront:
//   HBM bytes ~ n_tot * 16 * (2 + sum_j (nb_j - 1)/2) * (coalescing penalty),
//   plus a per-launch overhead for each tile level.
namespace {

double sweep_cost(const sylt_plan_s &p, const std::vector<int> &b)
{
    double R = 0.0;
    int levels = 1;
    for (int j = 0; j < p.M; ++j) {
        const int nb = (p.cdim[j] + b[j] - 1) / b[j];
        R += 0.5 * (nb - 1);
        levels += nb - 1;
    }
    // contiguous run of a tile row, in complex128 entries
    double run = 1;
    for (int j = 0; j < p.M; ++j) {
        run *= b[j];
        if (b[j] < p.cdim[j]) break;
    }
    const double penalty = std::max(1.0, 8.0 / run);
    const double bytes = (double)p.ntot * 16.0 * (2.0 + R) * penalty;
    return bytes / 4.0e12 + levels * 6.0e-6;
}

}  // namespace

void free_sweep_tables(SweepPlan &sp)
{
    if (sp.arena) (void)hipFree(sp.arena);
    sp.arena = nullptr;
    sp.d_desc = nullptr;
    sp.d_tiles = nullptr;
    sp.d_goff = nullptr;
    sp.d_code = nullptr;
    sp.d_llist = nullptr;
    sp.d_lloff = nullptr;
    sp.d_lanetab = nullptr;
    sp.d_cst = nullptr;
    sp.level_off.clear();
}

int plan_sweep(sylt_plan_s &p, const int *force_b)
{
    SweepPlan &sp = p.sweep;
    SweepDesc &sd = sp.desc;
    sd = SweepDesc{};
    sd.M = p.M;
    for (int k = 0; k < p.N; ++k)
        if (p.n[k] == 1) sd.singoff[sd.nsing++] = p.moff[k];
    const int M = p.M;
    const int bmax = sweep_max_partial_block();
    std::vector<int> b(M, 1);
    const size_t lds_cap = std::min<size_t>(max_lds_bytes(), 160 * 1024);
    auto tile_bytes = [&](const std::vector<int> &bb) {
        int64_t S = 1, td = 0;
        for (int j = 0; j < M; ++j) {
            S *= bb[j];
            td += (int64_t)bb[j] * bb[j];
        }
        return std::pair<int64_t, size_t>(S, (size_t)(S + td + 1) * sizeof(double2));
    };
    if (force_b) {
        // caller-chosen blocks: each a whole mode or at most the longest
        // partial block the pull loop holds, and the tile must fit the LDS
        for (int j = 0; j < M; ++j) {
            if (force_b[j] < 1 || force_b[j] > p.cdim[j]) return SYLT_E_INVALID_ARG;
            if (force_b[j] < p.cdim[j] && force_b[j] > bmax) return SYLT_E_UNSUPPORTED;
            b[j] = force_b[j];
        }
        auto tb = tile_bytes(b);
        if (tb.first > kSweepTileCap || tb.second > lds_cap) return SYLT_E_UNSUPPORTED;
    }
    // greedy: repeatedly take the move (a larger block on one mode) with the
    // best modelled gain that still fits the LDS budget
    for (; !force_b;) {
        const double cur = sweep_cost(p, b);
        double best_gain = 0.0;
        int best_j = -1, best_b = 0;
        for (int j = 0; j < M; ++j) {
            const int d = p.cdim[j];
            const int nb = (d + b[j] - 1) / b[j];
            for (int nbn = nb - 1; nbn >= 1; --nbn) {
                const int bn = (d + nbn - 1) / nbn;
                if (bn < d && bn > bmax) continue;
                std::vector<int> t = b;
                t[j] = bn;
                auto tb = tile_bytes(t);
                if (tb.first > kSweepTileCap || tb.second > lds_cap) continue;
                const double gain = (cur - sweep_cost(p, t)) / std::log2((double)bn / b[j]);
                if (gain > best_gain) {
                    best_gain = gain;
                    best_j = j;
                    best_b = bn;
                }
            }
        }
        if (best_j < 0) break;
        b[best_j] = best_b;
    }
    int64_t S = 1, ntiles = 1;
    int bitpos = 0, tdoff = 0, nll = 1, nlev = 1;
    for (int j = 0; j < M; ++j) {
        sd.d[j] = p.cdim[j];
        sd.s[j] = p.cstride[j];
        sd.b[j] = b[j];
        sd.nb[j] = (p.cdim[j] + b[j] - 1) / b[j];
        sd.ls[j] = (int)S;
        sd.bitw[j] = b[j] > 1 ? ilog2(b[j]) : 0;
        sd.bitoff[j] = bitpos;
        bitpos += sd.bitw[j];
        sd.tdoff[j] = tdoff;
        tdoff += b[j] * b[j];
        sd.moff[j] = p.moff[p.cmode[j]];
        S *= b[j];
        ntiles *= sd.nb[j];
        nll += b[j] - 1;
        nlev += sd.nb[j] - 1;
    }
    if (bitpos > 64 || ntiles > 0x7fffffff) return SYLT_E_UNSUPPORTED;
    sd.S = (int)S;
    sd.nll = nll;
    sd.tdiag = tdoff;
    sd.zero_slot = tdoff;  // one zero entry after the diagonal blocks
    sp.lds_bytes = (size_t)(S + tdoff + 1) * sizeof(double2);
    if (sp.lds_bytes > lds_cap) return SYLT_E_UNSUPPORTED;

    // local tables of the full tile
    std::vector<int64_t> goff(S);
    std::vector<uint64_t> code(S);
    std::vector<int> lev(S), llist(S), lloff(nll + 1, 0);
    for (int64_t t = 0; t < S; ++t) {
        int64_t rem = t, g = 0;
        uint64_t c = 0;
        int l = 0;
        for (int j = 0; j < M; ++j) {
            const int loc = (int)(rem % b[j]);
            rem /= b[j];
            g += (int64_t)loc * sd.s[j];
            c |= (uint64_t)loc << sd.bitoff[j];
            l += loc;
        }
        goff[t] = g;
        code[t] = c;
        lev[t] = l;
        lloff[l + 1]++;
    }
    for (int l = 0; l < nll; ++l) lloff[l + 1] += lloff[l];
    {
        std::vector<int> fill(lloff.begin(), lloff.end() - 1);
        for (int64_t t = 0; t < S; ++t) llist[fill[lev[t]]++] = (int)t;
    }
    // tiles ordered by block-index sum (tile level) and, within a level, in
    // Z-order (bit-interleaved block indices): consecutive tiles are
    // neighbours in every mode, so they share pull sources.  A mixed-radix
    // counter gives every tile id its level and Z key without divisions, and
    // an LSD radix sort orders the ids by (level, key).
    std::vector<int> tlev(ntiles);
    std::vector<uint64_t> key(ntiles, 0);
    sp.level_off.assign(nlev + 1, 0);
    int kbits = 0;
    {
        int maxnb = 1;
        for (int j = 0; j < M; ++j) maxnb = std::max(maxnb, sd.nb[j]);
        const int bits = std::max(1, ilog2(maxnb));
        if (M * bits <= 64) kbits = M * bits;  // otherwise keep the id order in a level
        std::vector<std::vector<uint64_t>> spread(M);
        for (int j = 0; j < M; ++j) {
            spread[j].assign(sd.nb[j], 0);
            if (kbits)
                for (int P = 0; P < sd.nb[j]; ++P)
                    for (int bit = 0; bit < bits; ++bit)
                        spread[j][P] |= (((uint64_t)P >> bit) & 1ull) << (bit * M + j);
        }
        std::vector<int> dig(M, 0);
        int l = 0;
        uint64_t k = 0;
        for (int64_t id = 0; id < ntiles; ++id) {
            tlev[id] = l;
            key[id] = k;
            sp.level_off[l + 1]++;
            for (int j = 0; j < M; ++j) {  // next id: increment the mixed-radix digits
                k -= spread[j][dig[j]];
                l -= dig[j];
                if (++dig[j] < sd.nb[j]) {
                    k += spread[j][dig[j]];
                    l += dig[j];
                    break;
                }
                dig[j] = 0;
            }
        }
    }
    for (int l = 0; l < nlev; ++l) sp.level_off[l + 1] += sp.level_off[l];
    std::vector<int> tiles(ntiles);
    {
        std::vector<int> order(ntiles), tmp(ntiles);
        for (int64_t id = 0; id < ntiles; ++id) order[id] = (int)id;
        constexpr int kDigit = 11;
        for (int shift = 0; shift < kbits; shift += kDigit) {
            std::vector<int64_t> cnt((1 << kDigit) + 1, 0);
            for (int64_t i = 0; i < ntiles; ++i) cnt[((key[order[i]] >> shift) & ((1 << kDigit) - 1)) + 1]++;
            for (int d = 0; d < (1 << kDigit); ++d) cnt[d + 1] += cnt[d];
            for (int64_t i = 0; i < ntiles; ++i)
                tmp[cnt[(key[order[i]] >> shift) & ((1 << kDigit) - 1)]++] = order[i];
            order.swap(tmp);
        }
        std::vector<int64_t> fill(sp.level_off.begin(), sp.level_off.end() - 1);
        for (int64_t i = 0; i < ntiles; ++i) tiles[fill[tlev[order[i]]]++] = order[i];
    }
    // per-lane packed local-solve work (one 32-bit word per lane and round)
    std::vector<int> lanetab(1, -1);
    sd.packed = 0;
    sd.rounds = 0;
    if (S <= (1 << 14) && bitpos <= 17) {
        std::vector<int> roff(nll + 1, 0);
        for (int l = 0; l < nll; ++l) {
            const int w = lloff[l + 1] - lloff[l];
            roff[l + 1] = roff[l] + (w + kSweepThreads - 1) / kSweepThreads;
        }
        if (roff[nll] <= kSweepMaxRounds) {
            lanetab.assign((size_t)roff[nll] * kSweepThreads, -1);
            for (int l = 0; l < nll; ++l)
                for (int idx = lloff[l]; idx < lloff[l + 1]; ++idx) {
                    const int k = idx - lloff[l];
                    const int r = roff[l] + k / kSweepThreads, lane = k % kSweepThreads;
                    const int t = llist[idx];
                    lanetab[(size_t)r * kSweepThreads + lane] = t | (int)(code[t] << 14);
                    sd.round_level[r] = l;
                }
            sd.packed = 1;
            sd.rounds = roff[nll];
        }
    }
    // pencil form of the local solve: one mode-0 pencil (loc_0 = 0 .. b_0-1)
    // per lane, the waves grouped by the pencil's index sum over the other
    // modes; it needs every group to fit the workgroup's waves.  A tile whose
    // last block along mode j >= 1 is short holds only the pencils with
    // loc_j < e_j; each such shape (a mask over modes 1..M-1) gets its own
    // packing, so a short tile's pencils fill fewer waves and the others skip
    // the entry work.
    sd.penc = 0;
    sd.pen_long = 0;
    for (int j = 1; j < M; ++j) sd.pen_long |= b[j] > 3;
    if (M >= 1 && M <= kSweepPencilModes && b[0] >= 4 && b[0] <= kSweepPencilMax && S <= (1 << 14) &&
        bitpos <= 17) {
        const int b0 = b[0];
        const int np = (int)(S / b0);
        const int nshape = 1 << (M - 1);
        std::vector<int> tab((size_t)nshape * kSweepThreads, -1);
        bool fits = true;
        for (int shape = 0; shape < nshape && fits; ++shape) {
            int e[kMaxModes];
            for (int j = 1; j < M; ++j)
                e[j] = (shape >> (j - 1)) & 1 ? p.cdim[j] - (sd.nb[j] - 1) * b[j] : b[j];
            std::vector<std::vector<int>> grp(nll - (b0 - 1));
            for (int pcl = 0; pcl < np; ++pcl) {
                const int64_t t0 = (int64_t)pcl * b0;
                bool in = true;
                for (int j = 1; j < M; ++j)
                    in = in && (int)((code[t0] >> sd.bitoff[j]) & ((1ull << sd.bitw[j]) - 1ull)) < e[j];
                if (in) grp[lev[t0]].push_back((int)t0 | (int)(code[t0] << 14));
            }
            int waves = 0;
            for (const auto &g : grp) waves += (int)((g.size() + 63) / 64);
            if (waves > kSweepThreads / 64) {
                fits = false;
                break;
            }
            int *ts = tab.data() + (size_t)shape * kSweepThreads;
            int w = 0;
            for (const auto &g : grp)
                for (size_t s0 = 0; s0 < g.size(); s0 += 64, ++w)
                    for (size_t i = s0; i < std::min(g.size(), s0 + 64); ++i)
                        ts[(size_t)w * 64 + (i - s0)] = g[i];
        }
        if (fits) {
            lanetab.swap(tab);
            sd.penc = 1;
            sd.packed = 0;
            sd.rounds = 0;
        }
    }
    // cross-section tables of the pull phase: for mode j, position c (the
    // mixed-radix digits over the other modes, fastest first) -> the local
    // entry with those digits and loc_j = 0
    std::vector<int> cst;
    for (int j = 0; j < M; ++j) {
        sd.csoff[j] = (int)cst.size();
        const int cs = (int)(S / b[j]);
        for (int c = 0; c < cs; ++c) {
            int rem = c, t0 = 0;
            for (int i = 0; i < M; ++i) {
                if (i == j || b[i] == 1) continue;
                t0 += (rem % b[i]) * sd.ls[i];
                rem /= b[i];
            }
            cst.push_back(t0);
        }
    }
    // every table in one device allocation, filled by one host-to-device copy
    std::vector<std::pair<const void *, size_t>> parts = {
        {&sd, sizeof(SweepDesc)},
        {goff.data(), S * sizeof(int64_t)},
        {code.data(), S * sizeof(uint64_t)},
        {lanetab.data(), lanetab.size() * sizeof(int)},
        {llist.data(), S * sizeof(int)},
        {lloff.data(), (nll + 1) * sizeof(int)},
        {tiles.data(), std::max<int64_t>(1, ntiles) * sizeof(int)},
        {cst.data(), cst.size() * sizeof(int)},
    };
    if (ntiles == 0) parts.back().first = nullptr;
    std::vector<size_t> off(parts.size());
    size_t total = 0;
    for (size_t i = 0; i < parts.size(); ++i) {
        off[i] = total;
        total += (parts[i].second + 255) & ~size_t(255);
    }
    std::vector<unsigned char> staging(total, 0);
    for (size_t i = 0; i < parts.size(); ++i)
        if (parts[i].first) memcpy(staging.data() + off[i], parts[i].first, parts[i].second);
    unsigned char *base = nullptr;
    SYLT_TRY(hipMalloc(&base, total));
    sp.arena = base;
    sp.d_desc = reinterpret_cast<SweepDesc *>(base + off[0]);
    sp.d_goff = reinterpret_cast<int64_t *>(base + off[1]);
    sp.d_code = reinterpret_cast<uint64_t *>(base + off[2]);
    sp.d_lanetab = reinterpret_cast<int *>(base + off[3]);
    sp.d_llist = reinterpret_cast<int *>(base + off[4]);
    sp.d_lloff = reinterpret_cast<int *>(base + off[5]);
    sp.d_tiles = reinterpret_cast<int *>(base + off[6]);
    sp.d_cst = reinterpret_cast<int *>(base + off[7]);
    SYLT_TRY(hipMemcpy(base, staging.data(), total, hipMemcpyHostToDevice));
    return SYLT_OK;
}

}  // namespace sylt

using namespace sylt;

namespace {

// hipFree waits for the device work that may still use the memory, so no
// explicit device synchronisation is needed here
void free_plan(sylt_plan_s *p)
{
    if (!p) return;
    if (p->arena) (void)hipFree(p->arena);
    if (p->dslo) (void)hipFree(p->dslo);
    if (p->dshi) (void)hipFree(p->dshi);
    free_sweep_tables(p->sweep);
    delete p;
}

// Shape bookkeeping and device allocation shared by both plan constructors.
int init_plan(sylt_plan_s *p, int N, const int64_t *n)
{
    SYLT_TRY(hipGetDevice(&p->device));
    p->N = N;
    p->n.assign(n, n + N);
    p->ntot = 1;
    p->moff.resize(N);
    p->mtotal = 0;
    int64_t stride = 1;
    for (int k = 0; k < N; ++k) {
        p->ntot *= n[k];
        p->moff[k] = p->mtotal;
        p->mtotal += n[k] * n[k];
        if (n[k] > 1) {
            p->cmode.push_back(k);
            p->cdim.push_back((int)n[k]);
            p->cstride.push_back(stride);
        }
        stride *= n[k];
    }
    p->M = (int)p->cmode.size();
    plan_passes(*p);
    int64_t maxt = 1;
    for (const PassDesc &pd : p->rpasses) maxt = std::max<int64_t>(maxt, pd.ntl * pd.ntr);
    for (const PassDesc &pd : p->mrpasses) maxt = std::max<int64_t>(maxt, pd.ntl * pd.ntr);
    p->scratch_bytes = (size_t)(std::max<int64_t>(2 * maxt, 4096) + 64) * sizeof(double);
    // the per-mode matrices, scratch and status words: one device allocation
    const size_t m16 = p->mtotal * sizeof(double2), m8 = p->mtotal * sizeof(float2);
    const size_t sizes[] = {m16, m16, m16, m16, m16, m16, m16, 3 * m16, 4 * sizeof(double2),
                            m8,  m8,  p->scratch_bytes, std::max(1, N) * sizeof(int)};
    size_t off[sizeof(sizes) / sizeof(sizes[0])], total = 0;
    for (size_t i = 0; i < sizeof(sizes) / sizeof(sizes[0]); ++i) {
        off[i] = total;
        total += (sizes[i] + 255) & ~size_t(255);
    }
    unsigned char *base = nullptr;
    SYLT_TRY(hipMalloc(&base, total));
    p->arena = base;
    p->dA = reinterpret_cast<double2 *>(base + off[0]);
    p->dU = reinterpret_cast<double2 *>(base + off[1]);
    p->dUh = reinterpret_cast<double2 *>(base + off[2]);
    p->dT = reinterpret_cast<double2 *>(base + off[3]);
    p->dTt = reinterpret_cast<double2 *>(base + off[4]);
    p->dTneg = reinterpret_cast<double2 *>(base + off[5]);
    p->dE = reinterpret_cast<double2 *>(base + off[6]);
    p->dEw = reinterpret_cast<double2 *>(base + off[7]);
    p->dEvo = reinterpret_cast<double2 *>(base + off[8]);
    p->dU32 = reinterpret_cast<float2 *>(base + off[9]);
    p->dUh32 = reinterpret_cast<float2 *>(base + off[10]);
    p->dScratch = reinterpret_cast<double *>(base + off[11]);
    p->dStatus = reinterpret_cast<int *>(base + off[12]);
    SYLT_TRY(hipMemset(p->dStatus, 0, std::max(1, N) * sizeof(int)));
    return plan_sweep(*p);
}

// Remark 1: if every T_k is diagonal to rounding (the Frobenius norm of its
// strictly upper part at most 16 n_k eps ||T_k||_F, as for normal A_k), the
// sweep becomes the Hadamard product with the inverse eigenvalue sums; build
// its two tables.
int plan_diagonal(sylt_plan_s *p, hipStream_t s)
{
    p->diagT = false;
    if (p->M == 0) return SYLT_OK;
    std::vector<double2> T(p->mtotal);
    SYLT_TRY(hipMemcpyAsync(T.data(), p->dT, p->mtotal * sizeof(double2), hipMemcpyDeviceToHost, s));
    SYLT_TRY(hipStreamSynchronize(s));
    for (int j = 0; j < p->M; ++j) {
        const int n = p->cdim[j];
        const double2 *Tj = T.data() + p->moff[p->cmode[j]];
        // the strictly upper part, as a whole (Frobenius norm), must be at the
        // level of the rounding of a backward-stable Schur factor: dropping it
        // is then a perturbation of T_k of the same order as that rounding
        double all2 = 0.0, off2 = 0.0;
        for (int c = 0; c < n; ++c)
            for (int r = 0; r <= c; ++r) {
                const double2 v = Tj[r + (int64_t)n * c];
                const double a2 = v.x * v.x + v.y * v.y;
                all2 += a2;
                if (r < c) off2 += a2;
            }
        if (std::sqrt(off2) > 16.0 * n * DBL_EPSILON * std::sqrt(all2)) return SYLT_OK;
    }
    // low table: the longest prefix of compressed modes with at most 2^16 entries
    int split = 0;
    int64_t lo = 1;
    while (split < p->M && lo * p->cdim[split] <= (1 << 16)) lo *= p->cdim[split++];
    p->dsplit = split;
    p->dlo = lo;
    p->dhi = p->ntot / lo;
    SYLT_TRY(hipMalloc(&p->dslo, p->dlo * sizeof(double2)));
    SYLT_TRY(hipMalloc(&p->dshi, p->dhi * sizeof(double2)));
    SYLT_TRY(launch_diag_tables(*p, s));
    p->diagT = true;
    return SYLT_OK;
}

// separation into the tail of the scratch, then one synchronisation
int finish_plan(sylt_plan_s *p, hipStream_t s, bool check_schur)
{
    SYLT_TRY(launch_prepare_factors(*p, s));
    double *d_sep = p->dScratch + (p->scratch_bytes / sizeof(double) - 8);
    SYLT_TRY(launch_separation(*p, d_sep, s));
    std::vector<int> st(p->N, 0);
    SYLT_TRY(hipMemcpyAsync(&p->sep, d_sep, sizeof(double), hipMemcpyDeviceToHost, s));
    SYLT_TRY(hipMemcpyAsync(st.data(), p->dStatus, p->N * sizeof(int), hipMemcpyDeviceToHost, s));
    SYLT_TRY(hipStreamSynchronize(s));
    if (check_schur)
        for (int k = 0; k < p->N; ++k)
            if (st[k]) return SYLT_E_NO_CONVERGENCE;
    if (!(p->sep > 0.0)) return SYLT_E_SINGULAR;
    return plan_diagonal(p, s);
}

int check_ptrs(int N, const double *const *P)
{
    if (!P) return SYLT_E_INVALID_ARG;
    for (int k = 0; k < N; ++k)
        if (!P[k]) return SYLT_E_INVALID_ARG;
    return SYLT_OK;
}

// Device-side phase timing for sylt_info: events recorded on the solve's
// stream at phase boundaries; inert when not requested.
class PhaseTimer {
  public:
    static constexpr int kMax = 8;
    PhaseTimer(bool on, hipStream_t s) : on_(on), s_(s)
    {
        for (int i = 0; on_ && i < kMax; ++i)
            if (hipEventCreate(&ev_[i]) != hipSuccess) {
                ok_ = false;
                n_ = i;
                on_ = false;
                return;
            }
        if (on_) n_ = kMax;
    }
    ~PhaseTimer()
    {
        for (int i = 0; i < n_; ++i) (void)hipEventDestroy(ev_[i]);
    }
    void reset() { used_ = 0; }
    void mark()
    {
        if (on_ && used_ < kMax && hipEventRecord(ev_[used_++], s_) != hipSuccess) ok_ = false;
    }
    // milliseconds between marks i and i + 1 (after the stream has synchronised)
    float span(int i)
    {
        float ms = 0.0f;
        if (!on_ || i + 1 >= used_) return 0.0f;
        if (hipEventElapsedTime(&ms, ev_[i], ev_[i + 1]) != hipSuccess) ok_ = false;
        return ms;
    }

  private:
    bool on_;
    hipStream_t s_;
    hipEvent_t ev_[kMax] = {};
    int n_ = 0, used_ = 0;
    bool ok_ = true;
};

// 2^-e for v in [2^e, 2^(e+1)), e clamped to [-1000, 1000]; 1 for v zero or
// not finite.  A power of two: applying it and its inverse rounds nothing.
double pow2_inverse(double v)
{
    if (!(v > 0.0) || !std::isfinite(v)) return 1.0;
    return std::ldexp(1.0, -std::max(-1000, std::min(1000, std::ilogb(v))));
}

int64_t mixed_workspace(const sylt_plan_s *p)
{
    const int64_t r64 = residual_pass_count(*p) > 1 ? p->ntot * (int64_t)sizeof(double2) : 0;
    return r64 + p->ntot * (int64_t)sizeof(float2) + 256;
}

}  // namespace

extern "C" {

int sylt_version(void) { return 200; }

const char *sylt_status_string(int code)
{
    switch (code) {
        case SYLT_OK: return "success";
        case SYLT_E_INVALID_ARG: return "invalid argument";
        case SYLT_E_SINGULAR: return "singular: an eigenvalue sum is zero";
        case SYLT_E_NO_CONVERGENCE: return "iteration did not converge";
        case SYLT_E_OUT_OF_MEMORY: return "out of device memory";
        case SYLT_E_DEVICE: return "HIP runtime error";
        case SYLT_E_UNSUPPORTED: return "outside the supported limits";
        case SYLT_E_WORKSPACE: return "workspace missing or too small";
        default: return "unknown status";
    }
}

int sylt_schur_factor_ex(int N, const int64_t *n, const double *const *A, int qr_iter_per_n,
                         void *stream, sylt_plan *out)
{
    if (!out) return SYLT_E_INVALID_ARG;
    *out = nullptr;
    int st = validate_shape(N, n);
    if (st) return st;
    if ((st = check_ptrs(N, A))) return st;
    sylt_plan_s *p = new (std::nothrow) sylt_plan_s();
    if (!p) return SYLT_E_OUT_OF_MEMORY;
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = init_plan(p, N, n);
    if (!st) {
        for (int k = 0; k < N && !st; ++k)
            st = status_of(hipMemcpyAsync(p->dA + p->moff[k], A[k], n[k] * n[k] * sizeof(double2),
                                          hipMemcpyDeviceToDevice, s));
    }
    if (!st)
        st = status_of(launch_schur(*p, qr_iter_per_n > 0 ? qr_iter_per_n : kSchurIterPerN, s));
    p->has_A = true;
    if (!st) st = finish_plan(p, s, true);
    if (st) {
        free_plan(p);
        return st;
    }
    *out = p;
    return SYLT_OK;
}

int sylt_schur_factor(int N, const int64_t *n, const double *const *A, void *stream, sylt_plan *out)
{
    return sylt_schur_factor_ex(N, n, A, 0, stream, out);
}

int sylt_plan_set_sweep_blocks(sylt_plan p, int M, const int *blocks)
{
    if (!p || !blocks || M != p->M) return SYLT_E_INVALID_ARG;
    if (M == 0) return SYLT_OK;
    // validate on a copy first so that a rejected request leaves the plan as it was
    for (int j = 0; j < M; ++j)
        if (blocks[j] < 1 || blocks[j] > p->cdim[j]) return SYLT_E_INVALID_ARG;
    SYLT_TRY(hipDeviceSynchronize());  // earlier calls may still read the old tables
    sylt::SweepPlan old = p->sweep;
    p->sweep = sylt::SweepPlan{};
    int st = plan_sweep(*p, blocks);
    if (st) {
        free_sweep_tables(p->sweep);
        p->sweep = old;
        return st;
    }
    free_sweep_tables(old);
    return SYLT_OK;
}

int sylt_plan_from_factors(int N, const int64_t *n, const double *const *A, const double *const *U,
                           const double *const *T, void *stream, sylt_plan *out)
{
    if (!out) return SYLT_E_INVALID_ARG;
    *out = nullptr;
    int st = validate_shape(N, n);
    if (st) return st;
    if ((st = check_ptrs(N, U)) || (st = check_ptrs(N, T))) return st;
    if (A && (st = check_ptrs(N, A))) return st;
    sylt_plan_s *p = new (std::nothrow) sylt_plan_s();
    if (!p) return SYLT_E_OUT_OF_MEMORY;
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = init_plan(p, N, n);
    for (int k = 0; k < N && !st; ++k) {
        const size_t bytes = n[k] * n[k] * sizeof(double2);
        st = status_of(hipMemcpyAsync(p->dU + p->moff[k], U[k], bytes, hipMemcpyDeviceToDevice, s));
        if (!st)
            st = status_of(hipMemcpyAsync(p->dT + p->moff[k], T[k], bytes, hipMemcpyDeviceToDevice, s));
        if (!st && A)
            st = status_of(hipMemcpyAsync(p->dA + p->moff[k], A[k], bytes, hipMemcpyDeviceToDevice, s));
    }
    p->has_A = A != nullptr;
    if (!st) st = finish_plan(p, s, false);
    if (st) {
        free_plan(p);
        return st;
    }
    *out = p;
    return SYLT_OK;
}

int sylt_plan_get_factors(sylt_plan p, int k, double *U, double *T, void *stream)
{
    if (!p || k < 0 || k >= p->N) return SYLT_E_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = p->n[k] * p->n[k] * sizeof(double2);
    if (U) SYLT_TRY(hipMemcpyAsync(U, p->dU + p->moff[k], bytes, hipMemcpyDeviceToDevice, s));
    if (T) SYLT_TRY(hipMemcpyAsync(T, p->dT + p->moff[k], bytes, hipMemcpyDeviceToDevice, s));
    return SYLT_OK;
}

int sylt_plan_separation(sylt_plan p, double *sep)
{
    if (!p || !sep) return SYLT_E_INVALID_ARG;
    *sep = p->sep;
    return SYLT_OK;
}

int sylt_plan_describe(sylt_plan p, char *buf, size_t len)
{
    if (!p || !buf || len == 0) return SYLT_E_INVALID_ARG;
    std::string s = "{\"N\":" + std::to_string(p->N) + ",\"n\":[";
    for (int k = 0; k < p->N; ++k) s += (k ? "," : "") + std::to_string(p->n[k]);
    s += "],\"ntot\":" + std::to_string(p->ntot);
    char sep[64];
    snprintf(sep, sizeof sep, "%.17g", p->sep);
    s += ",\"sep\":" + std::string(sep);
    auto passes = [&](const char *name, const std::vector<PassDesc> &v) {
        s += ",\"" + std::string(name) + "\":[";
        for (size_t i = 0; i < v.size(); ++i) {
            const PassDesc &d = v[i];
            s += (i ? "," : "") + std::string("{\"extents\":[");
            for (int q = 0; q < d.ng; ++q) s += (q ? "," : "") + std::to_string(d.gd[q]);
            s += "],\"Lin\":" + std::to_string(d.Lin) + ",\"G\":" + std::to_string(d.G) +
                 ",\"Rout\":" + std::to_string(d.Rout) + ",\"lb\":" + std::to_string(d.lb) +
                 ",\"rb\":" + std::to_string(d.rb) + ",\"tiles\":" + std::to_string(d.ntl * d.ntr) +
                 "}";
        }
        s += "]";
    };
    passes("transform_passes", p->passes);
    passes("residual_passes", p->residual_mfma ? p->mrpasses : p->rpasses);
    s += std::string(",\"residual_form\":\"") + (p->residual_mfma ? "mfma" : "valu") + "\"";
    const SweepDesc &sd = p->sweep.desc;
    int launches = 0;
    for (size_t l = 0; l + 1 < p->sweep.level_off.size(); ++l)
        launches += p->sweep.level_off[l + 1] > p->sweep.level_off[l];
    s += ",\"sweep\":{\"block\":[";
    for (int j = 0; j < sd.M; ++j) s += (j ? "," : "") + std::to_string(sd.b[j]);
    s += "],\"tile_entries\":" + std::to_string(sd.S) +
         ",\"tiles\":" + std::to_string(p->sweep.level_off.empty() ? 0 : p->sweep.level_off.back()) +
         ",\"tile_levels\":" + std::to_string(launches) + ",\"local_levels\":" + std::to_string(sd.nll) +
         ",\"local_solve\":\"" + (sd.penc ? "pencil" : sd.packed ? "packed" : "levels") + "\"" +
         ",\"diagonal\":" + (p->diagT ? "true" : "false") +
         ",\"lds_bytes\":" + std::to_string(p->sweep.lds_bytes) + "}}";
    const size_t n = std::min(len - 1, s.size());
    memcpy(buf, s.data(), n);
    buf[n] = '\0';
    return s.size() < len ? SYLT_OK : SYLT_E_INVALID_ARG;
}

int sylt_plan_destroy(sylt_plan p)
{
    if (!p) return SYLT_E_INVALID_ARG;
    free_plan(p);
    return SYLT_OK;
}

int64_t sylt_workspace_bytes(sylt_plan p, int precision)
{
    if (!p) return SYLT_E_INVALID_ARG;
    if (precision == SYLT_FP64) return (int64_t)std::max<size_t>(256, grad_A_workspace(*p) + 256);
    if (precision == SYLT_MIXED) return mixed_workspace(p);
    return SYLT_E_INVALID_ARG;
}

int sylt_transform(sylt_plan p, int dir, int precision, void *X, void *stream)
{
    if (!p || !X) return SYLT_E_INVALID_ARG;
    if (dir != SYLT_TO_SCHUR && dir != SYLT_FROM_SCHUR) return SYLT_E_INVALID_ARG;
    if (precision != SYLT_FP64 && precision != SYLT_MIXED) return SYLT_E_INVALID_ARG;
    return status_of(launch_transform(*p, dir, precision, X, static_cast<hipStream_t>(stream)));
}

int sylt_sweep(sylt_plan p, int op, int precision, void *CY, void *stream)
{
    if (!p || !CY) return SYLT_E_INVALID_ARG;
    if (op != SYLT_OP_N && op != SYLT_OP_C) return SYLT_E_INVALID_ARG;
    if (precision != SYLT_FP64 && precision != SYLT_MIXED) return SYLT_E_INVALID_ARG;
    return status_of(launch_sweep(*p, op, precision, CY, static_cast<hipStream_t>(stream)));
}

int sylt_residual(sylt_plan p, const double *B, const double *X, double *R, double *norms,
                  void *stream)
{
    if (!p || !B || !X || !R || !p->has_A) return SYLT_E_INVALID_ARG;
    if (p->M == 0) return SYLT_E_UNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *d_norms = p->dScratch + (p->scratch_bytes / sizeof(double) - 4);
    SYLT_TRY(launch_residual(*p, reinterpret_cast<const double2 *>(B),
                             reinterpret_cast<const double2 *>(X), reinterpret_cast<double2 *>(R),
                             nullptr, norms ? d_norms : nullptr, s));
    if (norms) {
        SYLT_TRY(hipMemcpyAsync(norms, d_norms, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        SYLT_TRY(hipStreamSynchronize(s));
    }
    return SYLT_OK;
}

int sylt_solve(sylt_plan p, const sylt_opts *o, const double *B, double *X, void *ws,
               size_t ws_bytes, void *stream, sylt_info *info)
{
    if (!p || !B || !X) return SYLT_E_INVALID_ARG;
    const int precision = o ? o->precision : SYLT_FP64;
    if (precision != SYLT_FP64 && precision != SYLT_MIXED) return SYLT_E_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2 *Xc = reinterpret_cast<double2 *>(X);
    const double2 *Bc = reinterpret_cast<const double2 *>(B);
    if (info) {
        info->status = SYLT_OK;
        info->iterations = 0;
        info->rel_residual = -1.0;
        info->sep = p->sep;
        info->ms_transform = info->ms_sweep = info->ms_residual = 0.0f;
    }
    // per-phase device times, only when info is requested
    PhaseTimer tm(info != nullptr, s);
    if (precision == SYLT_FP64) {
        tm.mark();
        SYLT_TRY(launch_transform_from(*p, SYLT_TO_SCHUR, Bc, Xc, s));
        tm.mark();
        SYLT_TRY(launch_sweep(*p, SYLT_OP_N, SYLT_FP64, Xc, s));
        tm.mark();
        SYLT_TRY(launch_transform(*p, SYLT_FROM_SCHUR, SYLT_FP64, Xc, s));
        tm.mark();
        if (info) {
            info->iterations = 1;
            SYLT_TRY(hipStreamSynchronize(s));
            info->ms_transform = tm.span(0) + tm.span(2);
            info->ms_sweep = tm.span(1);
        }
        return SYLT_OK;
    }
    // MIXED: iterative refinement with FP32 transforms.  B is read by every
    // residual, so X must not alias it.
    if (!p->has_A || p->M == 0 || Xc == Bc || o->max_iter < 1 || !(o->rtol >= 0.0))
        return SYLT_E_INVALID_ARG;
    if (!ws || (int64_t)ws_bytes < mixed_workspace(p)) return SYLT_E_WORKSPACE;
    char *w = static_cast<char *>(ws);
    double2 *R64 = nullptr;
    if (residual_pass_count(*p) > 1) {
        R64 = reinterpret_cast<double2 *>(w);
        w += p->ntot * sizeof(double2);
    }
    float2 *R32 = reinterpret_cast<float2 *>(w);
    double *d_norms = p->dScratch + (p->scratch_bytes / sizeof(double) - 4);
    // Every right-hand side enters FP32 times a power of two that brings it
    // near unit size (the first from max |B|, each residual from the size of
    // the right-hand side before it, which the refinement contracts by about
    // the FP32 accuracy), so neither B's own scale nor the shrinking residuals
    // reach FP32's overflow or subnormal range; the correction is unscaled
    // exactly in FP64.
    double bmax = 0.0;
    SYLT_TRY(launch_max_abs_c128(Bc, p->ntot, p->dScratch, d_norms + 2, s));
    SYLT_TRY(hipMemcpyAsync(&bmax, d_norms + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    SYLT_TRY(hipStreamSynchronize(s));
    double sc_in = pow2_inverse(bmax);  // scale of the right-hand side now in R32
    double sc_next = sc_in;              // scale of the next residual written to R32
    SYLT_TRY(launch_convert_c128_c64(R32, Bc, p->ntot, sc_in, s));
    int it = 0;
    double rel = -1.0;
    int st = SYLT_E_NO_CONVERGENCE;
    float ms_tr = 0.0f, ms_sw = 0.0f, ms_res = 0.0f;
    for (;;) {
        tm.reset();
        tm.mark();
        SYLT_TRY(launch_transform(*p, SYLT_TO_SCHUR, SYLT_MIXED, R32, s));
        tm.mark();
        SYLT_TRY(launch_sweep(*p, SYLT_OP_N, SYLT_MIXED, R32, s));
        tm.mark();
        SYLT_TRY(launch_transform(*p, SYLT_FROM_SCHUR, SYLT_MIXED, R32, s));
        tm.mark();
        SYLT_TRY(launch_axpy_c64(Xc, R32, p->ntot, it == 0, 1.0 / sc_in, s));
        ++it;
        tm.mark();
        SYLT_TRY(launch_residual(*p, Bc, Xc, R64, R32, d_norms, s, sc_next));
        tm.mark();
        double nrm[2];
        SYLT_TRY(hipMemcpyAsync(nrm, d_norms, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        SYLT_TRY(hipStreamSynchronize(s));
        sc_in = sc_next;
        sc_next = pow2_inverse(std::sqrt(nrm[0] / (double)p->ntot));
        ms_tr += tm.span(0) + tm.span(2);
        ms_sw += tm.span(1);
        ms_res += tm.span(4);
        rel = nrm[1] > 0.0 ? std::sqrt(nrm[0] / nrm[1]) : std::sqrt(nrm[0]);
        if (rel <= o->rtol) {
            st = SYLT_OK;
            break;
        }
        if (it >= o->max_iter || !std::isfinite(rel)) break;
    }
    if (info) {
        info->status = st;
        info->iterations = it;
        info->rel_residual = rel;
        info->ms_transform = ms_tr;
        info->ms_sweep = ms_sw;
        info->ms_residual = ms_res;
    }
    return st;
}

int64_t sylt_evolve_workspace_bytes(sylt_plan p)
{
    if (!p) return SYLT_E_INVALID_ARG;
    return 2 * p->ntot * (int64_t)sizeof(double2);
}

int sylt_evolve(sylt_plan p, double t, const double *B, const double *X0, double *X, void *ws,
                size_t ws_bytes, void *stream)
{
    if (!p || !B || !X0 || !X || !std::isfinite(t)) return SYLT_E_INVALID_ARG;
    if (!ws || (int64_t)ws_bytes < sylt_evolve_workspace_bytes(p)) return SYLT_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = p->ntot;
    double2 *Xc = reinterpret_cast<double2 *>(X);
    double2 *C = static_cast<double2 *>(ws);
    double2 *W = C + n;
    SYLT_TRY(launch_expm(*p, t, s));
    // C = U^*-chain(B) first, so that X may alias B
    SYLT_TRY(launch_transform_from(*p, SYLT_TO_SCHUR, reinterpret_cast<const double2 *>(B), C, s));
    // Y(0) = U^*-chain(X0), held in X
    SYLT_TRY(launch_transform_from(*p, SYLT_TO_SCHUR, reinterpret_cast<const double2 *>(X0), Xc, s));
    // W = sum_k T_k x_k Y(0) + C, as C - sum_k (-T_k) x_k Y(0)
    if (residual_pass_count(*p) > 0)
        SYLT_TRY(launch_residual_with(*p, p->dTneg, C, Xc, W, nullptr, nullptr, s));
    else  // every mode is a singleton: W = C + (sum a_k) Y(0)
        SYLT_TRY(launch_lincomb(W, C, Xc, p->dEvo + 2, n, s));
    // G = exp(t T_N) x_N ( ... exp(t T_1) x_1 W) - C, in X
    SYLT_TRY(launch_transform_with(*p, p->dE, W, s));
    SYLT_TRY(launch_lincomb(Xc, W, C, p->dEvo, n, s));
    // sum_k T_k x_k Y = G, then X(t) = U-chain(Y)
    SYLT_TRY(launch_sweep(*p, SYLT_OP_N, SYLT_FP64, Xc, s));
    SYLT_TRY(launch_transform(*p, SYLT_FROM_SCHUR, SYLT_FP64, Xc, s));
    return SYLT_OK;
}

int sylt_solve_backward_noalloc(sylt_plan p, const double *X, const double *GX, double *GB,
                                double *const *GA, void *stream)
{
    if (!p || !X || !GX || !GB) return SYLT_E_INVALID_ARG;
    void *scr = nullptr;
    size_t scr_bytes = 0;
    bool any = false;
    if (GA)
        for (int k = 0; k < p->N; ++k) any |= GA[k] != nullptr;
    if (any) {
        // the grad-A partial sums live in the fixed scratch; one n_k x n_k
        // matrix must fit (always true for n_k <= 256 and 8 MiB)
        SYLT_TRY(noalloc_scratch(&scr, &scr_bytes));
        for (int k = 0; k < p->N; ++k)
            if (GA[k] && (size_t)p->n[k] * p->n[k] * sizeof(double2) > scr_bytes)
                return SYLT_E_UNSUPPORTED;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2 *G = reinterpret_cast<double2 *>(GB);
    SYLT_TRY(launch_transform_from(*p, SYLT_TO_SCHUR, reinterpret_cast<const double2 *>(GX), G, s));
    SYLT_TRY(launch_sweep(*p, SYLT_OP_C, SYLT_FP64, G, s));
    SYLT_TRY(launch_transform(*p, SYLT_FROM_SCHUR, SYLT_FP64, G, s));
    if (any)
        SYLT_TRY(launch_grad_A(*p, G, reinterpret_cast<const double2 *>(X),
                               reinterpret_cast<double2 *const *>(GA), scr, scr_bytes, s));
    return SYLT_OK;
}

int sylt_solve_backward(sylt_plan p, const double *X, const double *GX, double *GB,
                        double *const *GA, void *ws, size_t ws_bytes, void *stream)
{
    if (!p || !X || !GX || !GB) return SYLT_E_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2 *G = reinterpret_cast<double2 *>(GB);
    SYLT_TRY(launch_transform_from(*p, SYLT_TO_SCHUR, reinterpret_cast<const double2 *>(GX), G, s));
    SYLT_TRY(launch_sweep(*p, SYLT_OP_C, SYLT_FP64, G, s));
    SYLT_TRY(launch_transform(*p, SYLT_FROM_SCHUR, SYLT_FP64, G, s));
    if (GA) {
        bool any = false;
        for (int k = 0; k < p->N; ++k) any |= GA[k] != nullptr;
        if (any) {
            if (!ws || ws_bytes < grad_A_workspace(*p)) return SYLT_E_WORKSPACE;
            SYLT_TRY(launch_grad_A(*p, G, reinterpret_cast<const double2 *>(X),
                                   reinterpret_cast<double2 *const *>(GA), ws, ws_bytes, s));
        }
    }
    return SYLT_OK;
}

}  // extern "C"
