// Handle creation: validation of the block hierarchy and the device tables
// (neighbours, coarse-fine ghost blocks, parents, covered octants, refluxing
// faces, dense multigrid levels).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <unordered_map>

#include "common.h"

namespace ohm {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

ohm_status fail(ohm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

std::mutex &capture_mutex()
{
    static std::mutex m;
    return m;
}

ohm_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(OHM_ERR_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
    return OHM_OK;
}

namespace {

inline int wrapi(int i, int n) { i %= n; return i < 0 ? i + n : i; }

inline uint64_t key3(int i, int j, int k)
{
    return ((uint64_t)(uint32_t)i << 42) | ((uint64_t)(uint32_t)j << 21) | (uint64_t)(uint32_t)k;
}

// i wrapped into [0, n); one conditional step for the usual offsets of a
// neighbour or a parent, the general remainder otherwise
inline int wrap1(int i, int n)
{
    if (i < 0) i += n;
    else if (i >= n) i -= n;
    return (i < 0 || i >= n) ? wrapi(i, n) : i;
}

// block coordinates -> index over a periodic box of blocks (-1 = none): a
// dense table when the box has at most 2^24 positions, a hash map otherwise
struct BoxIndex {
    int box[3] = {0, 0, 0};
    bool use_dense = false;
    std::vector<int> dense;
    std::unordered_map<uint64_t, int> sparse;
    void init(int b0, int b1, int b2)
    {
        box[0] = b0;
        box[1] = b1;
        box[2] = b2;
        const long long vol = (long long)b0 * b1 * b2;
        use_dense = vol <= (1LL << 24);
        if (use_dense) dense.assign((size_t)vol, -1);
    }
    size_t lin(int i, int j, int k) const { return (size_t)i + (size_t)box[0] * ((size_t)j + (size_t)box[1] * k); }
    int get(int i, int j, int k) const
    {
        i = wrap1(i, box[0]);
        j = wrap1(j, box[1]);
        k = wrap1(k, box[2]);
        if (use_dense) return dense[lin(i, j, k)];
        auto it = sparse.find(key3(i, j, k));
        return it == sparse.end() ? -1 : it->second;
    }
    bool has(int i, int j, int k) const { return get(i, j, k) >= 0; }
    // (i, j, k) inside the box; false if the position already has an index
    bool insert(int i, int j, int k, int v)
    {
        if (use_dense) {
            int &slot = dense[lin(i, j, k)];
            if (slot >= 0) return false;
            slot = v;
            return true;
        }
        return sparse.emplace(key3(i, j, k), v).second;
    }
};
using LevelMap = BoxIndex;   // block coords -> local block index of one level

bool coarsen_ok(const int n[3])
{
    return n[0] % 2 == 0 && n[1] % 2 == 0 && n[2] % 2 == 0 && n[0] >= 4 && n[1] >= 4 &&
           n[2] >= 4 && (long long)n[0] * n[1] * n[2] > 64;
}

// stream of the handle being built (uploads are ordered on it, then synchronised)
thread_local hipStream_t g_up_stream = nullptr;
// device bytes of the tables uploaded for the handle being built
thread_local size_t g_up_bytes = 0;

template <typename V>
ohm_status upload(V **dptr, const std::vector<V> &h)
{
    *dptr = nullptr;
    if (h.empty()) return OHM_OK;
    std::lock_guard<std::mutex> lock(capture_mutex());   // device work outside any captured stream
    OHM_HIP(hipMalloc((void **)dptr, sizeof(V) * h.size()));
    g_up_bytes += sizeof(V) * h.size();
    OHM_HIP(hipMemcpyAsync(*dptr, h.data(), sizeof(V) * h.size(), hipMemcpyHostToDevice, g_up_stream));
    OHM_HIP(hipStreamSynchronize(g_up_stream));
    return OHM_OK;
}

}  // namespace

static ohm_status build(ohm_hier *H, const ohm_problem_desc *probs, int nprob)
{
    H->nprob = nprob;
    H->probs.resize(nprob);
    // ---- validate and record each problem -------------------------------
    std::vector<std::vector<LevelMap>> maps(nprob);
    for (int p = 0; p < nprob; ++p) {
        const ohm_problem_desc &d = probs[p];
        ohm_prob_host &P = H->probs[p];
        if (d.nlevels < 1 || d.nlevels > OHM_MAX_LEVELS)
            return fail(OHM_ERR_ARG, "problem %d: nlevels %d outside 1..%d", p, d.nlevels, OHM_MAX_LEVELS);
        if (!(d.dx0 > 0.0)) return fail(OHM_ERR_ARG, "problem %d: dx0 must be positive", p);
        for (int a = 0; a < 3; ++a)
            if (d.base_blocks[a] < 1 || d.base_blocks[a] > 4096)
                return fail(OHM_ERR_ARG, "problem %d: base_blocks[%d] = %d", p, a, d.base_blocks[a]);
        P.nlevels = d.nlevels;
        P.dx0 = d.dx0;
        memcpy(P.bb, d.base_blocks, sizeof P.bb);
        maps[p].resize(d.nlevels);
        for (int l = 0; l < d.nlevels; ++l) {
            if (d.nblocks[l] < 1 || !d.block_ijk[l])
                return fail(OHM_ERR_ARG, "problem %d level %d: no blocks", p, l);
            LevelMap &M = maps[p][l];
            M.init(d.base_blocks[0] << l, d.base_blocks[1] << l, d.base_blocks[2] << l);
            P.blocks[l].assign(d.block_ijk[l], d.block_ijk[l] + 3 * (size_t)d.nblocks[l]);
            P.nb[l] = d.nblocks[l];
            for (int b = 0; b < d.nblocks[l]; ++b) {
                const int *q = &P.blocks[l][3 * b];
                for (int a = 0; a < 3; ++a)
                    if (q[a] < 0 || q[a] >= M.box[a])
                        return fail(OHM_ERR_LAYOUT, "problem %d level %d block %d: (%d,%d,%d) outside the box",
                                    p, l, b, q[0], q[1], q[2]);
                if (!M.insert(q[0], q[1], q[2], b))
                    return fail(OHM_ERR_LAYOUT, "problem %d level %d: duplicate block (%d,%d,%d)", p, l,
                                q[0], q[1], q[2]);
            }
        }
        long long full = (long long)d.base_blocks[0] * d.base_blocks[1] * d.base_blocks[2];
        if (d.nblocks[0] != full)
            return fail(OHM_ERR_LAYOUT, "problem %d: level 0 has %d blocks, the box needs %lld", p,
                        d.nblocks[0], full);
        // proper nesting: the 1-cell dilation of every level block and of every
        // face/edge neighbour position lies in level-(l-1) blocks
        for (int l = 1; l < d.nlevels; ++l) {
            const LevelMap &M = maps[p][l], &C = maps[p][l - 1];
            for (int b = 0; b < d.nblocks[l]; ++b) {
                const int *q = &P.blocks[l][3 * b];
                for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int nz_ = (dx != 0) + (dy != 0) + (dz != 0);
                    if (nz_ == 3) continue;
                    int n[3] = {q[0] + dx, q[1] + dy, q[2] + dz};
                    if (nz_ > 0 && M.has(n[0], n[1], n[2])) continue;
                    // coarse cells [4n-1, 4n+4] per axis -> coarse blocks
                    int lo[3], hi[3];
                    for (int a = 0; a < 3; ++a) {
                        lo[a] = (int)std::floor((4.0 * n[a] - 1) / 8.0);
                        hi[a] = (int)std::floor((4.0 * n[a] + 4) / 8.0);
                    }
                    for (int ck = lo[2]; ck <= hi[2]; ++ck)
                    for (int cj = lo[1]; cj <= hi[1]; ++cj)
                    for (int ci = lo[0]; ci <= hi[0]; ++ci)
                        if (!C.has(ci, cj, ck))
                            return fail(OHM_ERR_LAYOUT,
                                        "problem %d: level %d block (%d,%d,%d) is not properly nested in "
                                        "level %d (coarse block (%d,%d,%d) missing)",
                                        p, l, q[0], q[1], q[2], l - 1, wrapi(ci, C.box[0]),
                                        wrapi(cj, C.box[1]), wrapi(ck, C.box[2]));
                }
            }
        }
        // multigrid coarsenings of the base grid
        int n[3] = {8 * d.base_blocks[0], 8 * d.base_blocks[1], 8 * d.base_blocks[2]};
        int depth = 0;
        while (coarsen_ok(n)) {
            if (depth + 1 >= 16) break;
            for (int a = 0; a < 3; ++a) n[a] /= 2;
            ++depth;
            for (int a = 0; a < 3; ++a) P.dims[depth][a] = n[a];
        }
        P.min_level = -depth;
    }
    // ---- global level sizes -------------------------------------------------
    H->nlev = 0;
    H->min_level = 0;
    for (auto &P : H->probs) {
        H->nlev = std::max(H->nlev, P.nlevels);
        H->min_level = std::min(H->min_level, P.min_level);
    }
    H->nb_host.assign(H->nlev, 0);
    H->ng_host.assign(H->nlev, 0);
    H->blk_prob_host.assign(H->nlev, {});
    for (int l = 0; l < H->nlev; ++l)
        for (int p = 0; p < nprob; ++p) {
            ohm_prob_host &P = H->probs[p];
            if (l < P.nlevels) {
                P.boff[l] = H->nb_host[l];
                H->nb_host[l] += P.nb[l];
                for (int b = 0; b < P.nb[l]; ++b) H->blk_prob_host[l].push_back(p);
            } else {
                P.boff[l] = -1;
                P.nb[l] = 0;
            }
        }
    // dense levels: each problem's array starts on a 64-cell boundary (the
    // fused sweeps load aligned pairs), the gaps are never read or written
    for (int dd = 1; dd <= -H->min_level; ++dd) {
        long long c = 0;
        for (auto &P : H->probs) {
            if (-P.min_level >= dd) {
                P.doff[dd] = c;
                c += (long long)P.dims[dd][0] * P.dims[dd][1] * P.dims[dd][2];
                c = (c + 63) & ~63LL;
            } else {
                P.doff[dd] = -1;
            }
        }
        H->dense_cells[dd] = c;
    }
    // ---- AMR level tables ---------------------------------------------------
    for (int l = 0; l < H->nlev; ++l) {
        AmrLevelDev &L = H->amr[l];
        L.nb = H->nb_host[l];
        std::vector<int> nbr((size_t)L.nb * 27, NBR_NONE), prob(L.nb), ijk((size_t)L.nb * 3);
        std::vector<int> parent(L.nb, -1), octant(L.nb, 0), dmap;
        std::vector<int> gparent, goctant, gprob;
        std::vector<uint8_t> cov(L.nb, 0);
        if (l == 0) dmap.assign(L.nb, -1);
        int ng = 0;
        for (int p = 0; p < nprob; ++p) {
            ohm_prob_host &P = H->probs[p];
            if (l >= P.nlevels) continue;
            const LevelMap &M = maps[p][l];
            BoxIndex ghost_of;   // wrapped position -> ghost block
            ghost_of.init(M.box[0], M.box[1], M.box[2]);
            int lo3[3], hi3[3];
            for (int b = 0; b < P.nb[l]; ++b) {
                int gb = (int)P.boff[l] + b;
                const int *q = &P.blocks[l][3 * b];
                prob[gb] = p;
                for (int a = 0; a < 3; ++a) ijk[3 * gb + a] = q[a];
                for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int e = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
                    int n = M.get(q[0] + dx, q[1] + dy, q[2] + dz);
                    if (n >= 0) {
                        nbr[27 * (size_t)gb + e] = (int)P.boff[l] + n;
                        continue;
                    }
                    if ((dx != 0) + (dy != 0) + (dz != 0) == 3) {
                        // corners: only the fused two-halo sweep reads them; a
                        // ghost where the coarse cells its interpolation needs
                        // exist, else absent (the level then sweeps in halves)
                        bool ok = l >= 1;
                        for (int a = 0; a < 3 && ok; ++a) {
                            const int n = q[a] + (a == 0 ? dx : a == 1 ? dy : dz);
                            lo3[a] = (int)std::floor((4.0 * n - 1) / 8.0);
                            hi3[a] = (int)std::floor((4.0 * n + 4) / 8.0);
                        }
                        for (int ck = lo3[2]; ok && ck <= hi3[2]; ++ck)
                        for (int cj = lo3[1]; ok && cj <= hi3[1]; ++cj)
                        for (int ci = lo3[0]; ok && ci <= hi3[0]; ++ci)
                            ok = maps[p][l - 1].has(ci, cj, ck);
                        if (!ok) continue;
                    }
                    int w[3] = {wrapi(q[0] + dx, M.box[0]), wrapi(q[1] + dy, M.box[1]),
                                wrapi(q[2] + dz, M.box[2])};
                    int g = ghost_of.get(w[0], w[1], w[2]);
                    if (g < 0) {
                        g = ng++;
                        ghost_of.insert(w[0], w[1], w[2], g);
                        const LevelMap &C = maps[p][l - 1];
                        int pb = C.get(w[0] >> 1, w[1] >> 1, w[2] >> 1);
                        if (pb < 0) return fail(OHM_ERR_LAYOUT, "internal: ghost without parent");
                        gparent.push_back((int)P.boff[l - 1] + pb);
                        goctant.push_back((w[0] & 1) + 2 * (w[1] & 1) + 4 * (w[2] & 1));
                        gprob.push_back(p);
                    }
                    nbr[27 * (size_t)gb + e] = -1 - g;
                }
                if (l >= 1) {
                    const LevelMap &C = maps[p][l - 1];
                    int pb = C.get(q[0] >> 1, q[1] >> 1, q[2] >> 1);
                    parent[gb] = (int)P.boff[l - 1] + pb;
                    octant[gb] = (q[0] & 1) + 2 * (q[1] & 1) + 4 * (q[2] & 1);
                }
                if (l + 1 < P.nlevels) {
                    const LevelMap &F = maps[p][l + 1];
                    for (int o = 0; o < 8; ++o)
                        if (F.has(2 * q[0] + (o & 1), 2 * q[1] + ((o >> 1) & 1), 2 * q[2] + (o >> 2)))
                            cov[gb] |= (uint8_t)(1u << o);
                }
                if (l == 0) {
                    const int *dn = P.dims[1];
                    dmap[gb] = (int)(P.doff[1] + ((long long)(4 * q[2]) * dn[1] + 4 * q[1]) * dn[0] + 4 * q[0]);
                }
            }
        }
        L.ng = ng;
        H->ng_host[l] = ng;
        L.complete27 = std::all_of(nbr.begin(), nbr.end(), [](int v) { return v >= 0; });
        L.fused = std::all_of(nbr.begin(), nbr.end(), [](int v) { return v != NBR_NONE; });
        std::vector<double> ih2(nprob, 0.0), ih(nprob, 0.0);
        for (int p = 0; p < nprob; ++p)
            if (l < H->probs[p].nlevels) {
                double hh = H->probs[p].dx0 / (double)(1 << l);
                ih[p] = 1.0 / hh;
                ih2[p] = 1.0 / (hh * hh);
            }
        OHM_TRY(upload(&L.inv_h2, ih2));
        OHM_TRY(upload(&L.inv_h, ih));
        OHM_TRY(upload(&L.nbr, nbr));
        OHM_TRY(upload(&L.prob, prob));
        OHM_TRY(upload(&L.ijk, ijk));
        OHM_TRY(upload(&L.cov, cov));
        if (l >= 1) {
            OHM_TRY(upload(&L.parent, parent));
            OHM_TRY(upload(&L.octant, octant));
            OHM_TRY(upload(&L.gparent, gparent));
            OHM_TRY(upload(&L.goctant, goctant));
            OHM_TRY(upload(&L.gprob, gprob));
        }
        if (l == 0) OHM_TRY(upload(&L.dense_map, dmap));
    }
    // ---- refluxing faces: leaf cells of level l next to covered cells --------
    for (int l = 0; l + 1 < H->nlev; ++l) {
        std::vector<int> rf;
        for (int p = 0; p < nprob; ++p) {
            ohm_prob_host &P = H->probs[p];
            if (l + 1 >= P.nlevels) continue;
            const LevelMap &M = maps[p][l], &F = maps[p][l + 1];
            int box[3] = {M.box[0] * NB, M.box[1] * NB, M.box[2] * NB};
            // covered octants of every level-l block of the problem
            std::vector<uint8_t> cm(P.nb[l], 0);
            for (int b = 0; b < P.nb[l]; ++b) {
                const int *q = &P.blocks[l][3 * b];
                for (int o = 0; o < 8; ++o)
                    if (F.has(2 * q[0] + (o & 1), 2 * q[1] + ((o >> 1) & 1), 2 * q[2] + (o >> 2)))
                        cm[b] |= (uint8_t)(1u << o);
            }
            for (int b = 0; b < P.nb[l]; ++b) {
                const int *q = &P.blocks[l][3 * b];
                // masks of the block and its 6 face neighbours (0 if absent)
                uint8_t fm[3][2];
                bool any = cm[b] != 0;
                for (int d = 0; d < 3; ++d)
                    for (int s = 0; s < 2; ++s) {
                        int n[3] = {q[0], q[1], q[2]};
                        n[d] += s ? -1 : 1;
                        const int nb_ = M.get(n[0], n[1], n[2]);
                        fm[d][s] = nb_ >= 0 ? cm[nb_] : 0;
                        any |= fm[d][s] != 0;
                    }
                if (!any) continue;
                // is local cell (x,y,z), at most one coordinate outside 0..7, covered?
                auto covered = [&](int x, int y, int z) {
                    const int c[3] = {x, y, z};
                    uint8_t m = cm[b];
                    int l3[3] = {x, y, z};
                    for (int d = 0; d < 3; ++d) {
                        if (c[d] < 0) { m = fm[d][1]; l3[d] = c[d] + NB; }
                        else if (c[d] >= NB) { m = fm[d][0]; l3[d] = c[d] - NB; }
                    }
                    const int o = (l3[0] >> 2) + 2 * (l3[1] >> 2) + 4 * (l3[2] >> 2);
                    return ((m >> o) & 1) != 0;
                };
                for (int z = 0; z < NB; ++z)
                for (int y = 0; y < NB; ++y)
                for (int x = 0; x < NB; ++x) {
                    if (covered(x, y, z)) continue;
                    int ent[RF_INTS];
                    for (int t = 0; t < RF_INTS; ++t) ent[t] = -1;
                    int mask = 0;
                    for (int d = 0; d < 3; ++d)
                        for (int s = 0; s < 2; ++s) {
                            const int sg = s ? -1 : 1;
                            int lc[3] = {x, y, z};
                            lc[d] += sg;
                            if (!covered(lc[0], lc[1], lc[2])) continue;
                            const int f = 2 * d + s;
                            mask |= 1 << f;
                            // covered coarse cell Q (level-l global, wrapped)
                            int Q[3] = {q[0] * NB + x, q[1] * NB + y, q[2] * NB + z};
                            Q[d] += sg;
                            for (int a = 0; a < 3; ++a) Q[a] = wrapi(Q[a], box[a]);
                            const int fb = F.get(Q[0] >> 2, Q[1] >> 2, Q[2] >> 2);
                            // fine children of Q next to the face: along d the
                            // low child (2Q) when Q is above, the high one (2Q+1)
                            // when below; transverse the low child 2Q_t
                            int fl[3];
                            for (int a = 0; a < 3; ++a) fl[a] = 2 * Q[a] - NB * (Q[a] >> 2);
                            if (sg < 0) fl[d] += 1;
                            ent[3 + f] = (int)P.boff[l + 1] + fb;
                            ent[9 + f] = fl[0] + NB * (fl[1] + NB * fl[2]);
                        }
                    if (!mask) continue;
                    ent[0] = (int)P.boff[l] + b;
                    ent[1] = x + NB * (y + NB * z);
                    ent[2] = mask;
                    ent[15] = p;
                    rf.insert(rf.end(), ent, ent + RF_INTS);
                }
            }
        }
        const int nrf = (int)(rf.size() / RF_INTS);
        H->amr[l].nrf = nrf;
        OHM_TRY(upload(&H->amr[l].rf, rf));
        // face list and workgroup partition: whole entries per workgroup, at
        // most RF_WG_FACES faces
        std::vector<int> rff, rfs(nrf), rfw;
        int w_e0 = 0, w_f0 = 0;
        for (int e = 0; e <= nrf; ++e) {
            const int nf = e < nrf ? __builtin_popcount(rf[RF_INTS * e + 2]) : 0;
            const int cur = (int)rff.size() - w_f0;
            if (e == nrf || cur + nf > RF_WG_FACES) {
                if (e > w_e0) rfw.insert(rfw.end(), {w_e0, e - w_e0, w_f0, cur});
                w_e0 = e;
                w_f0 = (int)rff.size();
            }
            if (e == nrf) break;
            rfs[e] = (int)rff.size();
            for (int f = 0; f < 6; ++f)
                if ((rf[RF_INTS * e + 2] >> f) & 1) rff.push_back(8 * e + f);
        }
        H->amr[l].nrfw = (int)(rfw.size() / 4);
        OHM_TRY(upload(&H->amr[l].rff, rff));
        OHM_TRY(upload(&H->amr[l].rfs, rfs));
        OHM_TRY(upload(&H->amr[l].rfw, rfw));
    }
    // ---- dense levels ---------------------------------------------------------
    for (int dd = 1; dd <= -H->min_level; ++dd) {
        DenseLevelDev &D = H->dense[dd];
        D.ncells = (int)H->dense_cells[dd];
        std::vector<DenseProbDev> dp(nprob);
        std::vector<int> tiles, tiles_all, ft, ft_all, pt, pt_all;
        for (int p = 0; p < nprob; ++p) {
            ohm_prob_host &P = H->probs[p];
            DenseProbDev &q = dp[p];
            memset(&q, 0, sizeof q);
            if (-P.min_level < dd) continue;
            q.nx = P.dims[dd][0];
            q.ny = P.dims[dd][1];
            q.nz = P.dims[dd][2];
            q.active = (-P.min_level > dd) ? 1 : 0;
            q.off = P.doff[dd];
            double h = P.dx0 * (double)(1 << dd);
            q.inv_h2 = 1.0 / (h * h);
            int nc = q.nx * q.ny * q.nz;
            // fused sweeps on 8^3 tiles for even edges (the last tile of an
            // edge that is not a multiple of 8 wraps around), two half-sweeps
            // on 256-cell runs for an odd edge (its wrap would change colours)
            const bool tiled = q.nx % 2 == 0 && q.ny % 2 == 0 && q.nz % 2 == 0;
            const int ntiles = ((q.nx + NB - 1) / NB) * ((q.ny + NB - 1) / NB) * ((q.nz + NB - 1) / NB);
            for (int s = 0; s < nc; s += 256) {
                tiles_all.push_back(p);
                tiles_all.push_back(s);
                if (q.active) {
                    tiles.push_back(p);
                    tiles.push_back(s);
                }
                if (!tiled) {
                    pt_all.push_back(p);
                    pt_all.push_back(s);
                    if (q.active) {
                        pt.push_back(p);
                        pt.push_back(s);
                    }
                }
            }
            if (tiled)
                for (int t = 0; t < ntiles; ++t) {
                    ft_all.push_back(p);
                    ft_all.push_back(t);
                    if (q.active) {
                        ft.push_back(p);
                        ft.push_back(t);
                    }
                }
        }
        D.ntile = (int)tiles.size() / 2;
        D.ntile_all = (int)tiles_all.size() / 2;
        OHM_TRY(upload(&D.tiles, tiles));
        OHM_TRY(upload(&D.tiles_all, tiles_all));
        D.nftile = (int)ft.size() / 2;
        D.nftile_all = (int)ft_all.size() / 2;
        D.nptile = (int)pt.size() / 2;
        D.nptile_all = (int)pt_all.size() / 2;
        OHM_TRY(upload(&D.ftiles, ft));
        OHM_TRY(upload(&D.ftiles_all, ft_all));
        OHM_TRY(upload(&D.ptiles, pt));
        OHM_TRY(upload(&D.ptiles_all, pt_all));
        OHM_TRY(upload(&D.probs, dp));
    }
    // ---- scratch ---------------------------------------------------------------
    std::lock_guard<std::mutex> lock(capture_mutex());
    OHM_HIP(hipMalloc((void **)&H->d_scal, sizeof(double) * 4 * nprob));
    OHM_HIP(hipMalloc((void **)&H->d_norms, sizeof(double) * 8 * nprob));
    OHM_HIP(hipHostMalloc((void **)&H->h_dots, sizeof(double) * (8 + 2 * ITER_SLOTS + 6) * nprob, hipHostMallocDefault));
    size_t maxnb = 1;
    for (int l = 0; l < H->nlev; ++l) maxnb = std::max(maxnb, (size_t)H->nb_host[l]);
    H->part_cap = maxnb * 8 + 2 * (size_t)nprob * OHM_MAX_LEVELS + 64;
    OHM_HIP(hipMalloc((void **)&H->d_part, sizeof(double) * H->part_cap));
    H->table_bytes = g_up_bytes + sizeof(double) * (4 * (size_t)nprob + 8 * (size_t)nprob + H->part_cap);
    H->cinv_off.assign(nprob, -1);
    H->cinv_n.assign(nprob, 0);
    H->cinv_lamdt.assign(nprob, -1.0);
    H->cinv_prec.assign(nprob, -1);
    return OHM_OK;
}

static void free_all(ohm_hier *H)
{
    for (int l = 0; l < OHM_MAX_LEVELS; ++l) {
        AmrLevelDev &L = H->amr[l];
        void *ptrs[] = {L.nbr, L.prob, L.ijk, L.parent, L.octant, L.gparent, L.goctant, L.gprob,
                        L.cov, L.dense_map, L.rf, L.rff, L.rfs, L.rfw, L.inv_h2, L.inv_h};
        for (void *q : ptrs)
            if (q) (void)hipFree(q);
    }
    for (int d = 0; d < 16; ++d) {
        DenseLevelDev &D = H->dense[d];
        void *ptrs[] = {D.tiles, D.tiles_all, D.probs, D.ftiles, D.ftiles_all, D.ptiles, D.ptiles_all};
        for (void *q : ptrs)
            if (q) (void)hipFree(q);
    }
    void *ptrs[] = {H->d_scal, H->d_part, H->d_norms, H->d_coarse_inv, H->d_ring, H->d_coarse_eta, H->d_coarse_flags};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (H->h_dots) (void)hipHostFree(H->h_dots);
    if (H->stage_ev) (void)hipEventSynchronize(H->stage_ev);
    if (H->h_stage) (void)hipHostFree(H->h_stage);
    if (H->stage_ev) (void)hipEventDestroy(H->stage_ev);
    for (int i = 0; i < 64; ++i)
        if (H->ring_ev[i]) (void)hipEventDestroy(H->ring_ev[i]);
    for (auto &g : H->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (H->cap_stream) (void)hipStreamDestroy(H->cap_stream);
}

}  // namespace ohm

using namespace ohm;

extern "C" {

const char *ohm_last_error(void) { return g_err.c_str(); }

ohm_status ohm_hier_create(const ohm_problem_desc *probs, int32_t nprob, hipStream_t stream,
                           ohm_hier **out)
{
    if (!out) return fail(OHM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!probs || nprob < 1) return fail(OHM_ERR_ARG, "need at least one problem");
    ohm_hier *H = new (std::nothrow) ohm_hier();
    if (!H) return fail(OHM_ERR_NOMEM, "host allocation failed");
    // the host tables are built without the capture lock; each device
    // allocation and upload takes it
    g_up_stream = stream;
    g_up_bytes = 0;
    ohm_status st = build(H, probs, nprob);
    g_up_stream = nullptr;
    if (st != OHM_OK) {
        std::lock_guard<std::mutex> lock(capture_mutex());
        free_all(H);
        delete H;
        return st;
    }
    *out = H;
    return OHM_OK;
}

ohm_status ohm_hier_destroy(ohm_hier *h)
{
    if (!h) return OHM_OK;
    std::lock_guard<std::mutex> lock(capture_mutex());
    free_all(h);
    delete h;
    return OHM_OK;
}

ohm_status ohm_hier_device_bytes(const ohm_hier *h, size_t *bytes)
{
    if (!h || !bytes) return fail(OHM_ERR_ARG, "NULL argument");
    // tables and reduction scratch, plus what the first calls allocate: the
    // coefficient slots of the per-operation calls and the coarsest-grid
    // inverses of the step
    *bytes = h->table_bytes + sizeof(double) * 64 * (size_t)h->nprob + coarse_storage_bytes(h);
    return OHM_OK;
}

ohm_status ohm_hier_level_info(const ohm_hier *h, int32_t level, int64_t *nblocks, int64_t *ncells,
                               int64_t *nghost)
{
    if (!h) return fail(OHM_ERR_ARG, "handle is NULL");
    int64_t nb = 0, nc = 0, ng = 0;
    if (level >= 0) {
        if (level >= h->nlev) return fail(OHM_ERR_ARG, "level %d >= %d", level, h->nlev);
        nb = h->nb_host[level];
        nc = nb * NC;
        ng = h->ng_host[level];
    } else {
        if (level < h->min_level) return fail(OHM_ERR_ARG, "level %d below %d", level, h->min_level);
        nc = h->dense_cells[-level];
    }
    if (nblocks) *nblocks = nb;
    if (ncells) *ncells = nc;
    if (nghost) *nghost = ng;
    return OHM_OK;
}

ohm_status ohm_hier_problem_info(const ohm_hier *h, int32_t prob, int32_t level, int64_t *cell_offset,
                                 int32_t dims[3], int32_t *min_level)
{
    if (!h) return fail(OHM_ERR_ARG, "handle is NULL");
    if (prob < 0 || prob >= h->nprob) return fail(OHM_ERR_ARG, "problem %d out of range", prob);
    const ohm_prob_host &P = h->probs[prob];
    if (min_level) *min_level = P.min_level;
    int64_t off = -1;
    int32_t d3[3] = {0, 0, 0};
    if (level >= 0) {
        if (level < P.nlevels) {
            off = P.boff[level] * NC;
            for (int a = 0; a < 3; ++a) d3[a] = NB * (P.bb[a] << level);
        }
    } else if (level >= P.min_level) {
        off = P.doff[-level];
        for (int a = 0; a < 3; ++a) d3[a] = P.dims[-level][a];
    }
    if (cell_offset) *cell_offset = off;
    if (dims) memcpy(dims, d3, sizeof d3);
    return OHM_OK;
}

}  // extern "C"
