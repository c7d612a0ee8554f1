// Multilevel restricted additive Schwarz preconditioner on gfx950.
//
// Section 3.1: overlapping boxes Omega_i^delta (clipped at the domain
// boundary), subdomain matrices A_i = R_i^delta A R_i^delta^T factored by
// ILU(0) in local lexicographic order, applied as left-RAS (owned cells
// written once, no atomics), classical AS or right-RAS.
// Section 3.2: Algorithm 1 / the V-cycle preconditioner with
// Schwarz-Richardson smoothing, the Kaskade, additive and coarse-only
// compositions, the coarsest problem solved by Schwarz-preconditioned GMRES
// (Remark 2), first/second/third-order interpolation, restriction P^T and
// Galerkin coarse operators.
//
// GPU mapping: one workgroup per subdomain.  The triangular solves follow
// wavefront hyperplanes t = x + lb*y + lc*z (every lower stencil offset has a
// smaller t), which keeps the lexicographic elimination order of ILU(0) while
// running each hyperplane in parallel.  Factors are stored per subdomain in
// hyperplane order so each hyperplane is a contiguous, coalesced run; runs of
// hyperplanes are staged through LDS while the solution tile of the
// subdomain stays resident in LDS for both sweeps.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <type_traits>

#include "schwarz.h"

namespace nks {

static inline int nblk(int n, int t) { return (n + t - 1) / t; }

// ---------------------------------------------------------------- bf16 helpers
__host__ __device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);                                     // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
    uint32_t u = ((uint32_t)h) << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

template <typename FT> struct FTraits;
template <> struct FTraits<double> {
    __device__ static double get(const double *p, size_t i) { return p[i]; }
};
template <> struct FTraits<float> {
    __device__ static float get(const float *p, size_t i) { return p[i]; }
};
template <> struct FTraits<uint16_t> {
    __device__ static float get(const uint16_t *p, size_t i) { return from_bf16(p[i]); }
};

// ---------------------------------------------------------------- row templates (2D levels)
// stencil shapes: 0 = 5-point cross (lb 1), 1 = 5x5 box (lb 3), 2 = the
// 21-point stencil (5x5 without its corners, lb 3: the Galerkin product of
// the 5-point operator with second-order interpolation)
template <int BOX> struct RowStencil;
template <> struct RowStencil<0> {
    static constexpr int LB = 1, H = 1, NS = 4, NL = 2;
    // off-diagonal slots in increasing column order: (dx, dy)
    static constexpr int DX[NS] = {0, -1, 1, 0};
    static constexpr int DY[NS] = {-1, 0, 0, 1};
};
template <> struct RowStencil<1> {
    static constexpr int LB = 3, H = 8, NS = 24, NL = 12;
    static constexpr int DX[NS] = {-2, -1, 0, 1, 2, -2, -1, 0, 1, 2, -2, -1, 1, 2, -2, -1, 0, 1, 2, -2, -1, 0, 1, 2};
    static constexpr int DY[NS] = {-2, -2, -2, -2, -2, -1, -1, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2};
};
template <> struct RowStencil<2> {
    static constexpr int LB = 3, H = 8, NS = 20, NL = 10;
    static constexpr int DX[NS] = {-1, 0, 1, -2, -1, 0, 1, 2, -2, -1, 1, 2, -2, -1, 0, 1, 2, -1, 0, 1};
    static constexpr int DY[NS] = {-2, -2, -2, -1, -1, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 1, 1, 2, 2, 2};
};

// Per-cell factor runs of a row template: the lower run, then the upper
// run, each padded to whole 16-byte words of FT; where the two fit one word
// together (the 5-point cross in FP32 and BF16) they share it unpadded,
// which shrinks a box's LDS footprint by half or more.
template <int BOX, typename FT>
constexpr bool row_tight() {
    return RowStencil<BOX>::NS * sizeof(FT) <= 16;
}
template <int BOX, typename FT>
constexpr int row_lpad() {
    constexpr int PER = (int)(16 / sizeof(FT)), NL = RowStencil<BOX>::NL;
    return row_tight<BOX, FT>() ? NL : (NL + PER - 1) / PER * PER;
}
template <int BOX, typename FT>
constexpr int row_upad() {
    constexpr int PER = (int)(16 / sizeof(FT)), NU = RowStencil<BOX>::NS - RowStencil<BOX>::NL;
    return row_tight<BOX, FT>() ? NU : (NU + PER - 1) / PER * PER;
}
// padded run of a cell (both runs), whole 16-byte words
template <int BOX, typename FT>
constexpr int row_run() {
    return row_tight<BOX, FT>() ? (int)(16 / sizeof(FT)) : row_lpad<BOX, FT>() + row_upad<BOX, FT>();
}

// LDS stride of a cell's run in FT elements: an odd number of 16-byte
// words, so that the cells of one sweep step (ex - lb cells apart from lane
// to lane) fall in distinct LDS bank groups whenever ex - lb is odd
template <int BOX, typename FT>
constexpr int row_stride() {
    constexpr int R = row_run<BOX, FT>();
    return (R * sizeof(FT) / 16) % 2 ? R : R + (int)(16 / sizeof(FT));
}

// LDS stride of a cell's lower or upper run alone (the one-wavefront sweep
// holds one of them at a time), an odd number of 16-byte words as above
template <int BOX, typename FT>
constexpr int row_half_stride() {
    constexpr int PER = (int)(16 / sizeof(FT));
    constexpr int NL = RowStencil<BOX>::NL, NU = RowStencil<BOX>::NS - NL;
    constexpr int R = ((NL > NU ? NL : NU) + PER - 1) / PER * PER;
    return row_tight<BOX, FT>() ? row_stride<BOX, FT>() : ((R * sizeof(FT) / 16) % 2 ? R : R + PER);
}

// stencil index of every slot of the padded run (lower run, then upper
// run), from the 25 box slots of the level's stencil; -1 for absent slots
// and padding
template <int BOX, typename FT>
static void row_kmap(const std::vector<int> &slot, int (&kmap)[32]) {
    using S = RowStencil<BOX>;
    constexpr int NL = S::NL, NU = S::NS - S::NL;
    constexpr int NLP = row_lpad<BOX, FT>();
    for (int r = 0; r < 32; ++r) kmap[r] = -1;
    for (int q = 0; q < NL; ++q) kmap[q] = slot[(S::DX[q] + 2) + 5 * (S::DY[q] + 2)];
    for (int q = 0; q < NU; ++q) kmap[NLP + q] = slot[(S::DX[NL + q] + 2) + 5 * (S::DY[NL + q] + 2)];
}

// ---------------------------------------------------------------- host: partition
static void box_range(int n, int P, int q, int &lo, int &hi) {
    const int base = n / P, rem = n % P;
    lo = q * base + std::min(q, rem);
    hi = lo + base + (q < rem ? 1 : 0);
}

// wavefront coefficients: smallest lb, lc >= 1 with dx + lb dy + lc dz <= -1
// for every lower offset (lexicographically negative (dz, dy, dx))
static void wavefront(const Stencil &st, int &lb, int &lc) {
    lb = 1;
    lc = 1;
    for (int k = 0; k < st.K; ++k) {
        const int dx = st.off[3 * k], dy = st.off[3 * k + 1], dz = st.off[3 * k + 2];
        if (dz == 0 && dy < 0) lb = std::max(lb, (int)std::ceil((dx + 1.0) / (-dy)));
    }
    for (int k = 0; k < st.K; ++k) {
        const int dx = st.off[3 * k], dy = st.off[3 * k + 1], dz = st.off[3 * k + 2];
        if (dz < 0) lc = std::max(lc, (int)std::ceil((dx + lb * dy + 1.0) / (-dz)));
    }
}

static void build_partition(Level &L, const std::vector<std::array<int, 3>> &boxes, int delta, Alloc *al,
                            hipStream_t s, TileDims &geo) {
    const Space &S = *L.spp;
    const Stencil &st = L.fst;
    // the 3D register sweep holds the 7-point pattern only: with ILU(k) fill
    // the hyperplane kernels run there
    const bool nofill = L.fst.K == L.A->st.K;
    wavefront(st, L.lb, L.lc);
    int R = 0, Rz = 0;
    for (int k = 0; k < st.K; ++k) {
        R = std::max(R, (int)std::abs(st.off[3 * k]));
        R = std::max(R, (int)std::abs(st.off[3 * k + 1]));
        Rz = std::max(Rz, (int)std::abs(st.off[3 * k + 2]));
    }
    L.R = R;
    L.delta = delta;
    L.hsub.clear();
    L.hpart.clear();
    // first pass: boxes and maximum extents
    int mex = 1, mey = 1, mez = 1, minex = 1 << 30;
    for (int b = 0; b < S.B; ++b) {
        const Blk &k = S.hblk[b];
        const int P[3] = {std::min(boxes[b][0], k.nx), std::min(boxes[b][1], k.ny), std::min(boxes[b][2], k.nz)};
        const int n[3] = {k.nx, k.ny, k.nz};
        L.hpart.push_back({P[0], P[1], P[2], (int)L.hsub.size()});
        for (int qz = 0; qz < P[2]; ++qz)
            for (int qy = 0; qy < P[1]; ++qy)
                for (int qx = 0; qx < P[0]; ++qx) {
                    const int q[3] = {qx, qy, qz};
                    int lo[3], hi[3], elo[3], ehi[3];
                    for (int a = 0; a < 3; ++a) {
                        box_range(n[a], P[a], q[a], lo[a], hi[a]);
                        elo[a] = std::max(0, lo[a] - delta);
                        ehi[a] = std::min(n[a], hi[a] + delta);
                    }
                    SubDev sd{};
                    sd.blk = b;
                    sd.ex = ehi[0] - elo[0];
                    sd.ey = ehi[1] - elo[1];
                    sd.ez = ehi[2] - elo[2];
                    sd.ox = elo[0];
                    sd.oy = elo[1];
                    sd.oz = elo[2];
                    sd.lx0 = lo[0] - elo[0]; sd.lx1 = hi[0] - elo[0];
                    sd.ly0 = lo[1] - elo[1]; sd.ly1 = hi[1] - elo[1];
                    sd.lz0 = lo[2] - elo[2]; sd.lz1 = hi[2] - elo[2];
                    sd.next = sd.ex * sd.ey * sd.ez;
                    sd.gorg = k.off + elo[0] + k.nx * (elo[1] + k.ny * elo[2]);
                    sd.gnx = k.nx;
                    sd.gny = k.ny;
                    mex = std::max(mex, sd.ex);
                    minex = std::min(minex, sd.ex);
                    mey = std::max(mey, sd.ey);
                    mez = std::max(mez, sd.ez);
                    L.hsub.push_back(sd);
                }
    }
    geo.R = R;
    geo.Rz = Rz;
    geo.PX = mex + 2 * R;
    geo.PY = mey + 2 * R;
    geo.PZ = mez + 2 * Rz;
    const int tile = geo.PX * geo.PY * geo.PZ;
    L.max_tile = tile;
    // second pass: hyperplane order, maps
    std::vector<int> lvlptr, loc, inv, lexi, lexg;
    int fac = 0;
    L.max_next = 0;
    L.max_lvl = 0;
    L.max_nlev = 0;
    for (auto &sd : L.hsub) {
        sd.fac_off = fac;
        sd.lvl_off = (int)lvlptr.size();
        sd.inv_off = (int)inv.size();
        sd.nlev = (sd.ex - 1) + L.lb * (sd.ey - 1) + L.lc * (sd.ez - 1) + 1;
        std::vector<int> cnt(sd.nlev + 1, 0);
        for (int z = 0; z < sd.ez; ++z)
            for (int y = 0; y < sd.ey; ++y)
                for (int x = 0; x < sd.ex; ++x) cnt[x + L.lb * y + L.lc * z + 1]++;
        for (int t = 0; t < sd.nlev; ++t) cnt[t + 1] += cnt[t];
        for (int t = 0; t <= sd.nlev; ++t) lvlptr.push_back(cnt[t]);
        for (int t = 0; t < sd.nlev; ++t) L.max_lvl = std::max(L.max_lvl, cnt[t + 1] - cnt[t]);
        L.max_nlev = std::max(L.max_nlev, sd.nlev);
        std::vector<int> pos(cnt.begin(), cnt.end() - 1);
        std::vector<int> sloc(sd.next), slexi(sd.next);
        std::vector<int> sinv(tile, -1);
        for (int z = 0; z < sd.ez; ++z)
            for (int y = 0; y < sd.ey; ++y)
                for (int x = 0; x < sd.ex; ++x) {
                    const int t = x + L.lb * y + L.lc * z;
                    const int e = pos[t]++;
                    const int pidx = (x + R) + geo.PX * ((y + R) + geo.PY * (z + Rz));
                    sloc[e] = pidx;
                    slexi[e] = x + sd.ex * (y + sd.ey * z);
                    sinv[pidx] = e;
                }
        loc.insert(loc.end(), sloc.begin(), sloc.end());
        lexi.insert(lexi.end(), slexi.begin(), slexi.end());
        for (int e = 0; e < sd.next; ++e) lexg.push_back(sd.fac_off + slexi[e]);
        inv.insert(inv.end(), sinv.begin(), sinv.end());
        fac += sd.next;
        L.max_next = std::max(L.max_next, sd.next);
    }
    L.nsub = (int)L.hsub.size();
    L.next_total = fac;
    L.lvl_total = (int)lvlptr.size();
    L.inv_total = (int)inv.size();
    L.sub.upload(al, L.hsub, s);
    L.part.upload(al, L.hpart, s);
    L.lvlptr.upload(al, lvlptr, s);
    L.loc.upload(al, loc, s);
    L.inv.upload(al, inv, s);
    L.lexi.upload(al, lexi, s);
    L.lexg.upload(al, lexg, s);
    // 2D register-wavefront eligibility: rows fit one wavefront, reach <= 2
    L.rows2d = false;
    if (Rz == 0 && mey <= 64 && R <= 2) {
        std::vector<int> slot(25, -1);
        bool cross = st.K == 5;
        for (int k = 0; k < st.K; ++k) {
            const int dx = st.off[3 * k], dy = st.off[3 * k + 1];
            slot[(dx + 2) + 5 * (dy + 2)] = k;
            if (std::abs(dx) + std::abs(dy) > 1) cross = false;
        }
        bool corner = false;
        for (int k = 0; k < st.K; ++k)
            if (std::abs(st.off[3 * k]) == 2 && std::abs(st.off[3 * k + 1]) == 2) corner = true;
        const int box = cross ? 0 : (corner ? 1 : 2);
        // the sweep's cell arithmetic needs boxes at least LB wide
        if (minex >= (box == 0 ? RowStencil<0>::LB : RowStencil<1>::LB)) {
            L.box = box;
            L.slotmap.upload(al, slot, s);
            L.hslot = slot;
            L.rows2d = true;
        }
    }
    // 3D row sweep: the 7-point stencil, rows of at most 64 cells, at most
    // eight slabs of z planes with at most 64 (y, z) rows each
    L.rows3d = false;
    const int pzmin = 64 / std::max(mey, 1);
    if (nofill && Rz == 1 && R == 1 && st.K == 7 && mey <= 64 && mex <= 64 && (mez + pzmin - 1) / pzmin <= 8) {
        bool cross = true;
        for (int k = 0; k < st.K; ++k)
            if (std::abs(st.off[3 * k]) + std::abs(st.off[3 * k + 1]) + std::abs(st.off[3 * k + 2]) > 1) cross = false;
        if (cross) {
            auto find = [&](int dx, int dy, int dz) {
                for (int k = 0; k < st.K; ++k)
                    if (st.off[3 * k] == dx && st.off[3 * k + 1] == dy && st.off[3 * k + 2] == dz) return k;
                return -1;
            };
            L.hkmap3 = {find(0, 0, -1), find(0, -1, 0), find(-1, 0, 0), find(1, 0, 0), find(0, 1, 0), find(0, 0, 1)};
            L.rows3d = true;
            L.rows3d_multi = mey * mez > 64;
            L.rows3d_slabs = (mez + pzmin - 1) / pzmin;
        }
    }
    // stencil tables
    std::vector<int> lin(st.K);
    for (int k = 0; k < st.K; ++k)
        lin[k] = st.off[3 * k] + geo.PX * (st.off[3 * k + 1] + geo.PY * st.off[3 * k + 2]);
    L.lin_pad.upload(al, lin, s);
    std::map<std::tuple<int, int, int>, int> idx;
    for (int k = 0; k < st.K; ++k) idx[{st.off[3 * k], st.off[3 * k + 1], st.off[3 * k + 2]}] = k;
    std::vector<int> uptr(st.K + 1, 0), uk2, ut;
    for (int k = 0; k < st.K; ++k) {
        uptr[k] = (int)uk2.size();
        if (k < st.diag) {
            for (int k2 = st.diag + 1; k2 < st.K; ++k2) {
                auto it = idx.find({st.off[3 * k] + st.off[3 * k2], st.off[3 * k + 1] + st.off[3 * k2 + 1],
                                    st.off[3 * k + 2] + st.off[3 * k2 + 2]});
                if (it != idx.end()) {
                    uk2.push_back(k2);
                    ut.push_back(it->second);
                }
            }
        }
    }
    uptr[st.K] = (int)uk2.size();
    L.nupd = (int)uk2.size();
    L.max_upd = 0;
    for (int k = 0; k < st.K; ++k) L.max_upd = std::max(L.max_upd, uptr[k + 1] - uptr[k]);
    if (uk2.empty()) { uk2.push_back(0); ut.push_back(0); }
    L.upd_ptr.upload(al, uptr, s);
    L.upd_k2.upload(al, uk2, s);
    L.upd_t.upload(al, ut, s);
    L.err.alloc(al, 1);
    HIPC(hipMemsetAsync(L.err.p, 0, sizeof(int), s));
}

// ---------------------------------------------------------------- host: interpolation
// One direction of the interpolation from nc = ceil(nf/r) coarse cells to nf
// fine cells, coarse-to-fine ratio r.  Fine centre x_i = i + 1/2 in fine-cell
// units; coarse cell J covers fine cells rJ .. min(rJ + r, nf) - 1 and sits at
// their centroid.  Order 1: the parent cell (the first-order interpolation of
// Section 3.2).  Orders 2 and 3 work in the coarse index coordinate s(x),
// linear between consecutive centroids and continued one coarse spacing r
// past each end: order 2 is linear between the two centroids around x (one
// factor of the second-order interpolation), order 3 the cubic convolution
// W(s - J) over four coarse cells (the third-order interpolation).  Indices
// beyond the domain are clamped to the edge cell and their weights merged.
static double keys_kernel(double t) {
    t = std::fabs(t);
    if (t < 1.0) return (1.5 * t - 2.5) * t * t + 1.0;
    if (t < 2.0) return ((-0.5 * t + 2.5) * t - 4.0) * t + 2.0;
    return 0.0;
}

static void interp_weights(int nf, int order, int ratio, int i, std::vector<std::pair<int, double>> &out) {
    out.clear();
    const int nc = (nf + ratio - 1) / ratio;
    if (nf == 1) {
        out.push_back({0, 1.0});
        return;
    }
    std::vector<std::pair<int, double>> raw;
    if (order == 1) {
        raw.push_back({i / ratio, 1.0});
    } else {
        // centroids with a virtual one a coarse spacing past each end:
        // knot k of the list is coarse index k - 1
        std::vector<double> knot(nc + 2);
        for (int J = 0; J < nc; ++J) knot[J + 1] = 0.5 * (ratio * J + std::min(ratio * (J + 1), nf));
        knot[0] = knot[1] - ratio;
        knot[nc + 1] = knot[nc] + ratio;
        const double x = i + 0.5;
        // the knot interval [knot[k], knot[k+1]) holding x
        int k = (int)(std::upper_bound(knot.begin(), knot.end(), x) - knot.begin()) - 1;
        k = std::min(std::max(k, 0), nc);
        const double sx = (k - 1) + (x - knot[k]) / (knot[k + 1] - knot[k]);
        const int J0 = (int)std::floor(sx);
        const double t = sx - J0;
        if (order == 2) {
            raw.push_back({J0, 1.0 - t});
            raw.push_back({J0 + 1, t});
        } else {
            for (int l = -1; l <= 2; ++l) raw.push_back({J0 + l, keys_kernel(sx - (J0 + l))});
        }
    }
    for (auto &p : raw) {
        const int J = std::min(std::max(p.first, 0), nc - 1);
        bool merged = false;
        for (auto &q : out)
            if (q.first == J) { q.second += p.second; merged = true; }
        if (!merged) out.push_back({J, p.second});
    }
    std::sort(out.begin(), out.end());
    out.erase(std::remove_if(out.begin(), out.end(), [](const std::pair<int, double> &p) { return p.second == 0.0; }),
              out.end());
}

static void build_interp(Interp1 &ip, const std::vector<int> &nfs, int order, int ratio, Alloc *al, hipStream_t s) {
    ip.rcnt.clear(); ip.rj.clear(); ip.rw.clear();
    ip.ccnt.clear(); ip.ci.clear(); ip.cw.clear();
    ip.roff.clear(); ip.coff.clear();
    std::vector<std::pair<int, double>> w;
    // rows first; the column lists are the transposed rows, with a stride of
    // the longest column
    std::vector<std::vector<std::pair<int, double>>> cols;
    for (int nf : nfs) {
        const int nc = nf > 1 ? (nf + ratio - 1) / ratio : 1;
        const int r0 = (int)ip.rcnt.size(), c0 = (int)cols.size();
        ip.roff.push_back(r0);
        ip.coff.push_back(c0);
        ip.rcnt.resize(r0 + nf, 0);
        ip.rj.resize((size_t)(r0 + nf) * 4, 0);
        ip.rw.resize((size_t)(r0 + nf) * 4, 0.0);
        cols.resize(c0 + nc);
        for (int i = 0; i < nf; ++i) {
            interp_weights(nf, order, ratio, i, w);
            if (w.size() > 4) fail(NKS_EINVAL, "interpolation row with %zu entries", w.size());
            for (auto &p : w) {
                const int r = r0 + i;
                ip.rj[(size_t)r * 4 + ip.rcnt[r]] = p.first;
                ip.rw[(size_t)r * 4 + ip.rcnt[r]] = p.second;
                ip.rcnt[r]++;
                cols[c0 + p.first].push_back({i, p.second});
            }
        }
    }
    size_t cs = 1;
    for (auto &c : cols) cs = std::max(cs, c.size());
    ip.cs = (int)cs;
    ip.ccnt.assign(cols.size(), 0);
    ip.ci.assign(cols.size() * cs, 0);
    ip.cw.assign(cols.size() * cs, 0.0);
    for (size_t c = 0; c < cols.size(); ++c) {
        ip.ccnt[c] = (int)cols[c].size();
        for (size_t q = 0; q < cols[c].size(); ++q) {
            ip.ci[c * cs + q] = cols[c][q].first;
            ip.cw[c * cs + q] = cols[c][q].second;
        }
    }
    ip.d_rcnt.upload(al, ip.rcnt, s);
    ip.d_rj.upload(al, ip.rj, s);
    ip.d_rw.upload(al, ip.rw, s);
    ip.d_ccnt.upload(al, ip.ccnt, s);
    ip.d_ci.upload(al, ip.ci, s);
    ip.d_cw.upload(al, ip.cw, s);
    ip.d_roff.upload(al, ip.roff, s);
    ip.d_coff.upload(al, ip.coff, s);
}

// 1D coupling set S(o) = {J - I : P[f, I] != 0 and P[f + o, J] != 0}
static std::set<int> coupling_1d(const Interp1 &ip, const std::vector<int> &nfs, int o) {
    std::set<int> out;
    for (size_t b = 0; b < nfs.size(); ++b) {
        const int nf = nfs[b], r0 = ip.roff[b];
        for (int f = 0; f < nf; ++f) {
            const int g = f + o;
            if (g < 0 || g >= nf) continue;
            for (int a = 0; a < ip.rcnt[r0 + f]; ++a)
                for (int c = 0; c < ip.rcnt[r0 + g]; ++c)
                    out.insert(ip.rj[(size_t)(r0 + g) * 4 + c] - ip.rj[(size_t)(r0 + f) * 4 + a]);
        }
    }
    return out;
}

static void set_stencil(Stencil &st, std::vector<std::tuple<int, int, int>> offs, Alloc *al, hipStream_t s) {
    std::sort(offs.begin(), offs.end(), [](const std::tuple<int, int, int> &a, const std::tuple<int, int, int> &b) {
        return std::make_tuple(std::get<2>(a), std::get<1>(a), std::get<0>(a)) <
               std::make_tuple(std::get<2>(b), std::get<1>(b), std::get<0>(b));
    });
    st.K = (int)offs.size();
    if (st.K > MAXK) fail(NKS_EINVAL, "coarse stencil of %d points exceeds %d", st.K, MAXK);
    st.off.resize(3 * st.K);
    st.R = 0;
    for (int k = 0; k < st.K; ++k) {
        st.off[3 * k] = (int8_t)std::get<0>(offs[k]);
        st.off[3 * k + 1] = (int8_t)std::get<1>(offs[k]);
        st.off[3 * k + 2] = (int8_t)std::get<2>(offs[k]);
        if (std::get<0>(offs[k]) == 0 && std::get<1>(offs[k]) == 0 && std::get<2>(offs[k]) == 0) st.diag = k;
        st.R = std::max({st.R, std::abs(std::get<0>(offs[k])), std::abs(std::get<1>(offs[k])),
                         std::abs(std::get<2>(offs[k]))});
    }
    st.doff.upload(al, st.off, s);
}

// Factor stencil of ILU(k): the level-of-fill pattern of a row on an
// unbounded grid, where every row has the same pattern.  Eliminating the
// lower entry a (level la) of a row with the upper entry b (level lb) of
// row i+a gives the entry a+b the level la + lb + 1; the levels are iterated
// to their fixed point and the entries of level <= fill kept.  On a box the
// pattern is restricted to the cells inside it.  amap: factor entry ->
// operator entry, -1 for fill.
static void factor_stencil(const Stencil &op, int fill, Stencil &fst, std::vector<int> &amap, Alloc *al,
                           hipStream_t s) {
    using T3 = std::tuple<int, int, int>;
    auto key = [](const T3 &t) { return std::make_tuple(std::get<2>(t), std::get<1>(t), std::get<0>(t)); };
    const T3 zero{0, 0, 0};
    std::map<T3, int> lev;
    for (int k = 0; k < op.K; ++k) lev[{op.off[3 * k], op.off[3 * k + 1], op.off[3 * k + 2]}] = 0;
    for (bool changed = fill > 0; changed;) {
        changed = false;
        std::vector<std::pair<T3, int>> cur(lev.begin(), lev.end());
        for (auto &a : cur) {
            if (!(key(a.first) < key(zero))) continue;   // lower entries
            for (auto &b : cur) {
                if (!(key(zero) < key(b.first))) continue;   // upper entries of the neighbour's row
                const T3 c{std::get<0>(a.first) + std::get<0>(b.first), std::get<1>(a.first) + std::get<1>(b.first),
                           std::get<2>(a.first) + std::get<2>(b.first)};
                const int l = a.second + b.second + 1;
                if (l > fill) continue;
                auto it = lev.find(c);
                if (it == lev.end() || it->second > l) {
                    lev[c] = l;
                    changed = true;
                }
            }
        }
        if (lev.size() > (size_t)MAXK) fail(NKS_EINVAL, "ILU(%d) pattern exceeds %d points", fill, MAXK);
    }
    std::vector<T3> offs;
    for (auto &e : lev) offs.push_back(e.first);
    set_stencil(fst, offs, al, s);
    amap.assign(fst.K, -1);
    for (int k = 0; k < fst.K; ++k)
        for (int q = 0; q < op.K; ++q)
            if (op.off[3 * q] == fst.off[3 * k] && op.off[3 * q + 1] == fst.off[3 * k + 1] &&
                op.off[3 * q + 2] == fst.off[3 * k + 2])
                amap[k] = q;
}

// ---------------------------------------------------------------- kernels: ILU(0)
struct FacArgs {
    const SubDev *sub;
    const Blk *blk;
    const int *lvlptr, *loc, *inv, *lexi;
    const int *upd_ptr, *upd_k2, *upd_t, *lin;
    const double *A;      // operator coefficients, one array of N per operator entry
    const int *amap;      // factor entry -> operator entry (-1: fill, starts at zero)
    int N, NE, K, diag, PX, PY, R, Rz;
    const int8_t *off;
    double *w;            // K*NE workspace
    int *err;
};

// A_i rows of the extended cells, neighbours outside the box dropped
__global__ void k_ilu_fill(FacArgs a) {
    const SubDev sd = a.sub[blockIdx.x];
    const Blk bk = a.blk[sd.blk];
    for (int e = threadIdx.x; e < sd.next; e += blockDim.x) {
        const int lx = a.lexi[sd.fac_off + e];
        const int x = lx % sd.ex, y = (lx / sd.ex) % sd.ey, z = lx / (sd.ex * sd.ey);
        const int g = bk.off + (sd.ox + x) + bk.nx * ((sd.oy + y) + bk.ny * (sd.oz + z));
        for (int k = 0; k < a.K; ++k) {
            const int xx = x + a.off[3 * k], yy = y + a.off[3 * k + 1], zz = z + a.off[3 * k + 2];
            const bool in = xx >= 0 && xx < sd.ex && yy >= 0 && yy < sd.ey && zz >= 0 && zz < sd.ez;
            const int ka = a.amap[k];
            a.w[(size_t)k * a.NE + sd.fac_off + e] = (in && ka >= 0) ? a.A[(size_t)ka * a.N + g] : 0.0;
        }
    }
}

// IKJ elimination row by row in hyperplane order.  Row i, for each lower
// neighbour k in increasing column order: l_ik = a_ik / u_kk, then
// a_ij -= l_ik u_kj for the j in row i's pattern.  Rows of one hyperplane are
// independent; their lower neighbours lie on earlier hyperplanes.
__global__ void k_ilu_factor(FacArgs a) {
    extern __shared__ double smem_f[];
    const SubDev sd = a.sub[blockIdx.x];
    double *row = smem_f + (size_t)threadIdx.x * a.K;
    int *lp = reinterpret_cast<int *>(smem_f + (size_t)blockDim.x * a.K);
    for (int t = threadIdx.x; t <= sd.nlev; t += blockDim.x) lp[t] = a.lvlptr[sd.lvl_off + t];
    __syncthreads();
    for (int t = 0; t < sd.nlev; ++t) {
        const int p0 = lp[t], p1 = lp[t + 1];
        for (int el = p0 + threadIdx.x; el < p1; el += blockDim.x) {
            const size_t e = (size_t)sd.fac_off + el;
            for (int k = 0; k < a.K; ++k) row[k] = a.w[(size_t)k * a.NE + e];
            const int lc = a.loc[e];
            for (int kl = 0; kl < a.diag; ++kl) {
                if (row[kl] == 0.0) continue;
                const int e2l = a.inv[sd.inv_off + lc + a.lin[kl]];
                if (e2l < 0) continue;   // neighbour outside the box (only reachable after a bad pivot)
                const size_t e2 = (size_t)sd.fac_off + e2l;
                const double l = row[kl] / a.w[(size_t)a.diag * a.NE + e2];
                row[kl] = l;
                for (int q = a.upd_ptr[kl]; q < a.upd_ptr[kl + 1]; ++q)
                    row[a.upd_t[q]] -= l * a.w[(size_t)a.upd_k2[q] * a.NE + e2];
            }
            if (!(row[a.diag] != 0.0) || !isfinite(row[a.diag])) atomicOr(a.err, 1);
            for (int k = 0; k < a.K; ++k) a.w[(size_t)k * a.NE + e] = row[k];
        }
        __syncthreads();
    }
}

// The same elimination with the whole box in LDS (2D boxes): the rows of
// A_i (gathered from the operator as k_ilu_fill does), the padded-tile
// inverse map, the level pointers and the elimination tables are staged
// once; the hyperplanes are eliminated in place and the factors written back.
// MAXL / MAXQ bound the lower stencil entries and the updates per lower entry
// (5-point cross: 2 / 1; 7-point: 3 / 3; 5x5 box: 12 / 12).  The row loop is branch-free: a
// lower neighbour's index and pivot are read up front (earlier hyperplanes
// are final), and the update lists are padded by repeating their last entry,
// which rewrites the same value.
// LDS: K*max_next doubles, then ints: tile + (nlev+1) + K + (K+1) + 2*nupd + next.
template <int MAXL, int MAXQ>
__global__ void __launch_bounds__(256) k_ilu_factor_lds(FacArgs a, int max_next, int tile, int nupd) {
    extern __shared__ double smem_f[];
    const SubDev sd = a.sub[blockIdx.x];
    const Blk bk = a.blk[sd.blk];
    const int K = a.K, n = sd.next, diag = a.diag;
    double *W = smem_f;
    int *inv = reinterpret_cast<int *>(W + (size_t)K * max_next);
    int *lp = inv + tile;
    int *lin = lp + (sd.nlev + 1);
    int *uptr = lin + K;
    int *ut = uptr + (K + 1);
    int *uk = ut + nupd;
    int *loc = uk + nupd;
    for (int i = threadIdx.x; i < tile; i += blockDim.x) inv[i] = a.inv[sd.inv_off + i];
    for (int i = threadIdx.x; i <= sd.nlev; i += blockDim.x) lp[i] = a.lvlptr[sd.lvl_off + i];
    for (int i = threadIdx.x; i < K; i += blockDim.x) lin[i] = a.lin[i];
    for (int i = threadIdx.x; i <= K; i += blockDim.x) uptr[i] = a.upd_ptr[i];
    for (int i = threadIdx.x; i < nupd; i += blockDim.x) {
        ut[i] = a.upd_t[i];
        uk[i] = a.upd_k2[i];
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) loc[i] = a.loc[sd.fac_off + i];
    // rows of A_i: neighbours outside the box dropped
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int lx = a.lexi[sd.fac_off + e];
        const int x = lx % sd.ex, y = (lx / sd.ex) % sd.ey, z = lx / (sd.ex * sd.ey);
        const int g = bk.off + (sd.ox + x) + bk.nx * ((sd.oy + y) + bk.ny * (sd.oz + z));
        for (int k0 = 0; k0 < K; k0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = min(k0 + u, K - 1);
                const int xx = x + a.off[3 * k], yy = y + a.off[3 * k + 1], zz = z + a.off[3 * k + 2];
                const bool in = xx >= 0 && xx < sd.ex && yy >= 0 && yy < sd.ey && zz >= 0 && zz < sd.ez;
                const int ka = a.amap[k];
                v[u] = (in && ka >= 0) ? a.A[(size_t)max(ka, 0) * a.N + g] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < K) W[(size_t)(k0 + u) * n + e] = v[u];
        }
    }
    __syncthreads();
    for (int t = 0; t < sd.nlev; ++t) {
        for (int el = lp[t] + threadIdx.x; el < lp[t + 1]; el += blockDim.x) {
            const int lc = loc[el];
            int e2v[MAXL];
            double piv[MAXL];
#pragma unroll
            for (int kl = 0; kl < MAXL; ++kl) e2v[kl] = inv[lc + lin[min(kl, diag - 1)]];
#pragma unroll
            for (int kl = 0; kl < MAXL; ++kl) piv[kl] = W[(size_t)diag * n + max(e2v[kl], 0)];
#pragma unroll
            for (int kl = 0; kl < MAXL; ++kl) {
                if (kl < diag) {
                    const double aik = W[(size_t)kl * n + el];
                    const int e2 = max(e2v[kl], 0);
                    // e2v < 0: neighbour outside the box (only reachable after a bad pivot)
                    const bool on = aik != 0.0 && e2v[kl] >= 0;
                    const double l = on ? aik / piv[kl] : 0.0;
                    if (on) W[(size_t)kl * n + el] = l;
                    const int q0 = uptr[kl], cnt = uptr[kl + 1] - q0;
                    if (cnt > 0) {
                        int tq[MAXQ], kq[MAXQ];
#pragma unroll
                        for (int q = 0; q < MAXQ; ++q) {
                            const int qq = q0 + min(q, cnt - 1);
                            tq[q] = ut[qq];
                            kq[q] = uk[qq];
                        }
                        double uv[MAXQ], rv[MAXQ];
#pragma unroll
                        for (int q = 0; q < MAXQ; ++q) {
                            uv[q] = W[(size_t)kq[q] * n + e2];
                            rv[q] = W[(size_t)tq[q] * n + el];
                        }
#pragma unroll
                        for (int q = 0; q < MAXQ; ++q)
                            if (on) W[(size_t)tq[q] * n + el] = rv[q] - l * uv[q];
                    }
                }
            }
            const double d = W[(size_t)diag * n + el];
            if (!(d != 0.0) || !isfinite(d)) atomicOr(a.err, 1);
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < K * n; i += blockDim.x) {
        const int k = i / n, e = i - k * n;
        a.w[(size_t)k * a.NE + sd.fac_off + e] = W[i];
    }
}

// storage precision: off-diagonals in FT, 1/u_ii in DT
template <typename FT, typename DT>
__global__ void k_ilu_store(const double *w, int NE, int K, int diag, FT *f, DT *invd, const int *perm) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)NE) return;
    const size_t d = perm ? (size_t)perm[e] : e;
    for (int k = 0; k < K; ++k) {
        const double v = w[(size_t)k * NE + e];
        if (k == diag) {
            invd[d] = (DT)(1.0 / v);
        } else {
            if constexpr (sizeof(FT) == 2) f[(size_t)k * NE + d] = to_bf16((float)v);
            else f[(size_t)k * NE + d] = (FT)v;
        }
    }
}

// ---------------------------------------------------------------- staging helpers
constexpr int STAGE_U = 16;   // independent loads in flight per thread while staging

// dst[i] = src[i] for i < n, by the whole workgroup, STAGE_U loads in flight
template <typename T, typename S>
__device__ __forceinline__ void stage_copy(T *dst, const S *src, int n) {
    const int bs = blockDim.x;
    for (int i0 = threadIdx.x; i0 < n; i0 += STAGE_U * bs) {
        S v[STAGE_U];
#pragma unroll
        for (int u = 0; u < STAGE_U; ++u) {
            const int i = i0 + u * bs;
            if (i < n) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < STAGE_U; ++u) {
            const int i = i0 + u * bs;
            if (i < n) dst[i] = (T)v[u];
        }
    }
}

// K segments of n elements: dst[k*dstride + j] = src[k*sstride + j]
template <typename T, typename S>
__device__ __forceinline__ void stage_copy_k(T *dst, int dstride, const S *src, size_t sstride, int K, int n) {
    const int bs = blockDim.x, tot = K * n;
    for (int i0 = threadIdx.x; i0 < tot; i0 += STAGE_U * bs) {
        S v[STAGE_U];
#pragma unroll
        for (int u = 0; u < STAGE_U; ++u) {
            const int i = i0 + u * bs;
            if (i < tot) v[u] = src[(size_t)(i / n) * sstride + (i % n)];
        }
#pragma unroll
        for (int u = 0; u < STAGE_U; ++u) {
            const int i = i0 + u * bs;
            if (i < tot) dst[(i / n) * dstride + (i % n)] = (T)v[u];
        }
    }
}

// ---------------------------------------------------------------- kernel: subdomain solves
// LDS layout of the apply kernel: solution tile, stencil offsets, staged
// coefficients, staged 1/u_ii, staged tile positions (16-byte aligned parts).
struct ApplyLds {
    size_t lin, lp, cf, cd, cl, total;
};
__host__ __device__ __forceinline__ size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }
__host__ __device__ __forceinline__ ApplyLds apply_lds(size_t vt, size_t ft, size_t dt, int tile, int ncmax,
                                                       int cap, int maxlev) {
    ApplyLds L;
    L.lin = al16(vt * (size_t)tile);
    L.lp = al16(L.lin + sizeof(int) * MAXK);
    L.cf = al16(L.lp + sizeof(int) * (size_t)(maxlev + 1));
    L.cd = al16(L.cf + ft * (size_t)ncmax * cap);
    L.cl = al16(L.cd + dt * (size_t)cap);
    L.total = al16(L.cl + sizeof(int) * (size_t)cap);
    return L;
}

struct ApplyArgs {
    const SubDev *sub;
    const Blk *blk;
    const int *lvlptr, *loc, *lexi, *lin;
    int maxlev;           // most hyperplanes of any subdomain
    const void *F;        // K*NE off-diagonal factors (FT)
    const void *invd;     // NE (DT)
    int NE, K, diag, PX, PY, PZ, R, Rz, tile;
    const double *r;
    double *z, *zext;
    const int *mask;
    unsigned long long *units;   // profiled launches: swept extended / owned cells
    int variant, accumulate, cap;
    int lin7[7];          // 7-point kernel: tile offsets of the stencil entries
};

// One subdomain per workgroup: gather R_i^delta r into the LDS tile, forward
// sweep with the unit lower factor, backward sweep with the upper factor,
// then write the owned cells (left-RAS) or the whole box (AS / right-RAS).
// NC = 3: the 7-point stencil (three lower and three upper terms, tile
// offsets from the kernel arguments); NC = 0: any stencil, terms in blocks
// of eight.
template <typename FT, typename VT, typename DT, int NC>
__global__ void __launch_bounds__(256) k_ras_apply(ApplyArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const SubDev sd = a.sub[blockIdx.x];
    if (a.mask && !a.mask[sd.blk]) return;
    if (a.units && threadIdx.x == 0) {
        // spread over PROF_UNIT_SLOTS counter pairs, so the workgroups of a
        // launch do not queue on one address
        unsigned long long *u = a.units + 2 * (blockIdx.x % PROF_UNIT_SLOTS);
        atomicAdd(u, (unsigned long long)sd.next);
        atomicAdd(u + 1, (unsigned long long)((sd.lx1 - sd.lx0) * (sd.ly1 - sd.ly0) * (sd.lz1 - sd.lz0)));
    }
    const Blk bk = a.blk[sd.blk];
    const int ncl = NC ? NC : a.diag, ncu = NC ? NC : a.K - a.diag - 1;
    const int ncmax = ncl > ncu ? ncl : ncu;
    const ApplyLds lay = apply_lds(sizeof(VT), sizeof(FT), sizeof(DT), a.tile, ncmax, a.cap, a.maxlev);
    VT *tile = reinterpret_cast<VT *>(smem);
    int *lin = reinterpret_cast<int *>(smem + lay.lin);
    int *lp = reinterpret_cast<int *>(smem + lay.lp);
    FT *cf = reinterpret_cast<FT *>(smem + lay.cf);      // ncmax * cap
    DT *cd = reinterpret_cast<DT *>(smem + lay.cd);      // cap
    int *cl = reinterpret_cast<int *>(smem + lay.cl);    // cap
    const FT *F = reinterpret_cast<const FT *>(a.F);
    const DT *ID = reinterpret_cast<const DT *>(a.invd);
    for (int k = threadIdx.x; k < a.K; k += blockDim.x) lin[k] = a.lin[k];
    for (int t = threadIdx.x; t <= sd.nlev; t += blockDim.x) lp[t] = a.lvlptr[sd.lvl_off + t];
    for (int i = threadIdx.x; i < a.tile; i += blockDim.x) tile[i] = (VT)0;
    __syncthreads();
    // gather R_i^delta r (right-RAS: R_i^0 r, zero on the overlap)
    for (int c0 = threadIdx.x; c0 < sd.next; c0 += STAGE_U * blockDim.x) {
        double v[STAGE_U];
#pragma unroll
        for (int u = 0; u < STAGE_U; ++u) {
            const int c = c0 + u * blockDim.x;
            if (c < sd.next) {
                const int x = c % sd.ex, y = (c / sd.ex) % sd.ey, z = c / (sd.ex * sd.ey);
                const int g = bk.off + (sd.ox + x) + bk.nx * ((sd.oy + y) + bk.ny * (sd.oz + z));
                v[u] = a.r[g];
            }
        }
#pragma unroll
        for (int u = 0; u < STAGE_U; ++u) {
            const int c = c0 + u * blockDim.x;
            if (c < sd.next) {
                const int x = c % sd.ex, y = (c / sd.ex) % sd.ey, z = c / (sd.ex * sd.ey);
                const bool own = x >= sd.lx0 && x < sd.lx1 && y >= sd.ly0 && y < sd.ly1 && z >= sd.lz0 && z < sd.lz1;
                tile[(x + a.R) + a.PX * ((y + a.R) + a.PY * (z + a.Rz))] =
                    (VT)((a.variant == NKS_RIGHT_RAS && !own) ? 0.0 : v[u]);
            }
        }
    }
    __syncthreads();
    const size_t fo = sd.fac_off;
    // forward: y_i = r_i - sum_{lower k} L_ik y_k
    for (int t0 = 0; t0 < sd.nlev;) {
        const int c0 = lp[t0];
        int t1 = t0 + 1;
        while (t1 < sd.nlev && lp[t1 + 1] - c0 <= a.cap) ++t1;
        const int c1 = lp[t1];
        stage_copy_k(cf, a.cap, F + fo + c0, (size_t)a.NE, ncl, c1 - c0);
        stage_copy(cl, a.loc + fo + c0, c1 - c0);
        __syncthreads();
        for (int t = t0; t < t1; ++t) {
            for (int e = lp[t] + threadIdx.x; e < lp[t + 1]; e += blockDim.x) {
                const int le = e - c0;
                const int p = cl[le];
                VT v = tile[p];
                if constexpr (NC > 0) {
                    VT cv[NC], tv[NC];
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        cv[k] = (VT)FTraits<FT>::get(cf, (size_t)k * a.cap + le);
                        tv[k] = tile[p + a.lin7[k]];
                    }
#pragma unroll
                    for (int k = 0; k < NC; ++k) v -= cv[k] * tv[k];
                    tile[p] = v;
                    continue;
                }
                // eight terms at a time, every load issued before the first
                // product (a padded term adds an exact zero)
                for (int k0 = 0; k0 < ncl; k0 += 8) {
                    VT cv[8], tv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int k = min(k0 + u, ncl - 1);
                        const VT c = (VT)FTraits<FT>::get(cf, (size_t)k * a.cap + le);
                        tv[u] = tile[p + lin[k]];
                        cv[u] = k0 + u < ncl ? c : (VT)0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) v -= cv[u] * tv[u];
                }
                tile[p] = v;
            }
            __syncthreads();
        }
        t0 = t1;
    }
    // backward: z_i = (y_i - sum_{upper k} U_ik z_k) / u_ii
    for (int t1 = sd.nlev; t1 > 0;) {
        const int c1 = lp[t1];
        int t0 = t1 - 1;
        while (t0 > 0 && c1 - lp[t0 - 1] <= a.cap) --t0;
        const int c0 = lp[t0];
        stage_copy_k(cf, a.cap, F + (size_t)(a.diag + 1) * a.NE + fo + c0, (size_t)a.NE, ncu, c1 - c0);
        stage_copy(cd, ID + fo + c0, c1 - c0);
        stage_copy(cl, a.loc + fo + c0, c1 - c0);
        __syncthreads();
        for (int t = t1 - 1; t >= t0; --t) {
            for (int e = lp[t] + threadIdx.x; e < lp[t + 1]; e += blockDim.x) {
                const int le = e - c0;
                const int p = cl[le];
                VT v = tile[p];
                if constexpr (NC > 0) {
                    VT cv[NC], tv[NC];
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        cv[k] = (VT)FTraits<FT>::get(cf, (size_t)k * a.cap + le);
                        tv[k] = tile[p + a.lin7[NC + 1 + k]];
                    }
#pragma unroll
                    for (int k = 0; k < NC; ++k) v -= cv[k] * tv[k];
                    tile[p] = v * (VT)cd[le];
                    continue;
                }
                for (int k0 = 0; k0 < ncu; k0 += 8) {
                    VT cv[8], tv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int k = min(k0 + u, ncu - 1);
                        const VT c = (VT)FTraits<FT>::get(cf, (size_t)k * a.cap + le);
                        tv[u] = tile[p + lin[a.diag + 1 + k]];
                        cv[u] = k0 + u < ncu ? c : (VT)0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) v -= cv[u] * tv[u];
                }
                tile[p] = v * (VT)cd[le];
            }
            __syncthreads();
        }
        t1 = t0;
    }
    // scatter
    if (a.variant == NKS_LEFT_RAS) {
        const int ox = sd.lx1 - sd.lx0, oy = sd.ly1 - sd.ly0, oz = sd.lz1 - sd.lz0;
        const int no = ox * oy * oz;
        // WB cells per thread per pass: with accumulation, every load of z
        // is issued before the first store
        constexpr int WB = 8;
        const int bs = blockDim.x;
        for (int c0 = threadIdx.x; c0 < no; c0 += WB * bs) {
            int g[WB];
            double v[WB];
#pragma unroll
            for (int u = 0; u < WB; ++u) {
                const int c = min(c0 + u * bs, no - 1);
                const int x = sd.lx0 + c % ox, y = sd.ly0 + (c / ox) % oy, z = sd.lz0 + c / (ox * oy);
                g[u] = bk.off + (sd.ox + x) + bk.nx * ((sd.oy + y) + bk.ny * (sd.oz + z));
                v[u] = (double)tile[(x + a.R) + a.PX * ((y + a.R) + a.PY * (z + a.Rz))];
            }
            if (a.accumulate) {
#pragma unroll
                for (int u = 0; u < WB; ++u) v[u] += a.z[g[u]];
            }
#pragma unroll
            for (int u = 0; u < WB; ++u)
                if (c0 + u * bs < no) a.z[g[u]] = v[u];
        }
    } else {
        for (int c = threadIdx.x; c < sd.next; c += blockDim.x) {
            const int x = c % sd.ex, y = (c / sd.ex) % sd.ey, z = c / (sd.ex * sd.ey);
            a.zext[fo + c] = (double)tile[(x + a.R) + a.PX * ((y + a.R) + a.PY * (z + a.Rz))];
        }
    }
}


// ---------------------------------------------------------------- kernel: 2D register wavefront
// One wavefront per subdomain, lane = row y of the extended box.  At step t
// lane y handles cell x = t - LB*y (the hyperplane order), so every lower
// neighbour (x+dx, y+dy) was produced by lane y+dy exactly
// -(dx + LB*dy) steps earlier.  Each lane keeps its last H outputs in a
// register ring and reads the rows below / above through DPP lane shifts;
// only the factor coefficients and the right-hand side come from LDS.
__device__ __forceinline__ float lane_shr(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_shl(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_shr(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_shl(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
// the value of lane src_addr / 4 (a lane permute through the LDS crossbar)
__device__ __forceinline__ float lane_from(float v, int src_addr) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src_addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_from(double v, int src_addr) {
    const int lo = __builtin_amdgcn_ds_bpermute(src_addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src_addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

struct RowsArgs {
    const SubDev *sub;
    const void *F;        // K*NE off-diagonal factors (FT), lexicographic per subdomain
    const void *invd;     // NE (DT)
    int NE;
    const double *r;
    double *z, *zext;
    const int *mask;
    unsigned long long *units;   // profiled launches: swept extended / owned cells
    int variant, accumulate;
    int kmap[32];         // slot of the padded per-cell run -> stencil index (-1: absent or padding)
};

// coefficients of one cell: N consecutive FT values, in 16-byte words, or
// one 8- or 4-byte word (the runs of the 5-point cross in FP32 and BF16)
template <typename FT, typename VT, int N>
__device__ __forceinline__ void load_run(const FT *p, VT (&out)[N]) {
    constexpr int B = (int)(N * sizeof(FT));
    static_assert(B % 16 == 0 || B == 8 || B == 4, "runs are whole 16-byte words, or one smaller word");
    auto put = [&](const FT *f, int k0, int cnt) {
#pragma unroll
        for (int k = 0; k < cnt; ++k) {
            if constexpr (sizeof(FT) == 2) out[k0 + k] = (VT)from_bf16(f[k]);
            else out[k0 + k] = (VT)f[k];
        }
    };
    if constexpr (B == 8) {
        const uint2 u = *reinterpret_cast<const uint2 *>(p);
        put(reinterpret_cast<const FT *>(&u), 0, N);
    } else if constexpr (B == 4) {
        const uint32_t u = *reinterpret_cast<const uint32_t *>(p);
        put(reinterpret_cast<const FT *>(&u), 0, N);
    } else {
        constexpr int W = B / 16, PER = (int)(16 / sizeof(FT));
        const uint4 *q = reinterpret_cast<const uint4 *>(p);
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint4 u = q[w];
            put(reinterpret_cast<const FT *>(&u), w * PER, PER);
        }
    }
}

// (x, y) of cell c of a box ex wide, by a float reciprocal: exact for
// c < 2^16 and ex <= 64, where (c + 1/2) / ex stays 1/128 off integers
__device__ __forceinline__ int row_of(int c, float inv_ex) { return (int)(((float)c + 0.5f) * inv_ex); }

// Steps per unrolled sweep iteration (the register ring length) and the
// guard cells on each side of the sweeps' LDS arrays: the padded steps of
// the last iteration and the look-ahead block read up to RU + RU/2 - 1
// cells past either end of a box.
__host__ __device__ constexpr int rows_unroll(int box) { return box == 0 ? 16 : 8; }
__host__ __device__ constexpr int rows_pad(int box) { return rows_unroll(box) + rows_unroll(box) / 2; }
struct RowsLds {
    size_t rv, cf, id, total;
};
__host__ __device__ inline RowsLds rows_lds(size_t vt, size_t ft, size_t dt, int cs, int pad, size_t n) {
    RowsLds L;
    L.rv = 0;
    L.cf = al16(vt * (n + 1 + 2 * pad));
    L.id = L.cf + al16(ft * cs * (n + 2 * pad));
    L.total = L.id + al16(dt * (n + 2 * pad));
    return L;
}

// Every instruction of the sweeping wavefront costs an issue slot (one
// wavefront per SIMD), so the step loop keeps only the arithmetic, the LDS
// traffic and the lane shifts: the cell of step t is cb + t, which stays in
// the box for every t when the box is at least LB cells wide (steps outside
// a row's range read a neighbouring row's cell and are masked; rows past
// the box repeat the last row), stores of masked steps go to a spare slot,
// and the stencil map arrives in the kernel arguments.  The upper factors and 1/u_ii are
// staged by the other wavefronts while the forward sweep runs.  The
// cross-stencil form in FP32 / BF16 is held to five wavefronts per SIMD: its
// boxes then fit five to a CU in registers as in LDS.
template <typename FT, typename VT, typename DT, int BOX, int NT>
__global__ void __launch_bounds__(NT, (BOX == 0 && NT == 256 && sizeof(VT) == 4) ? 5 : 1) k_ras_rows(RowsArgs a) {
    using S = RowStencil<BOX>;
    constexpr int NS = S::NS, NL = S::NL, NU = NS - NL, LB = S::LB;
    constexpr int PER = (int)(16 / sizeof(FT));
    constexpr int NLP = row_lpad<BOX, FT>(), NUP = row_upad<BOX, FT>();
    constexpr int NSP = NLP + NUP;   // padded run per cell: lower run, then upper run
    // NT = 256: one wavefront sweeps while the other three stage the upper
    // runs beside the lower ones; NT = 64: the lower runs are staged, the
    // forward sweep runs, then the upper runs take their place in LDS
    constexpr bool ONE = NT == 64;
    constexpr int CS = ONE ? row_half_stride<BOX, FT>() : row_stride<BOX, FT>();   // LDS stride of a cell
    constexpr int UOFF = ONE ? 0 : NLP;   // the upper run's offset in a cell's LDS slot
    constexpr int RU = rows_unroll(BOX);   // unroll = ring length (>= the deepest history used)
    constexpr int PAD = rows_pad(BOX);
    static_assert(NT == 256 || NT == 64, "one or four wavefronts");
    // cells per staging thread per pass: a 36x36 cross-stencil box in one
    // pass, so its loads pay the memory latency once
    constexpr int CPT = ONE ? 2 : (BOX == 0 ? 6 : 2);
    constexpr int CPU = 2;           // the same for the upper runs (staged during the forward sweep)
    constexpr int NST = NLP;         // slots staged before the forward sweep
    static_assert(NSP <= 32, "stencil map fits the argument block");
    extern __shared__ __align__(16) unsigned char smem[];
    const SubDev sd = a.sub[blockIdx.x];
    if (a.mask && !a.mask[sd.blk]) return;
    if (a.units && threadIdx.x == 0) {
        // spread over PROF_UNIT_SLOTS counter pairs, so the workgroups of a
        // launch do not queue on one address
        unsigned long long *u = a.units + 2 * (blockIdx.x % PROF_UNIT_SLOTS);
        atomicAdd(u, (unsigned long long)sd.next);
        atomicAdd(u + 1, (unsigned long long)((sd.lx1 - sd.lx0) * (sd.ly1 - sd.ly0) * (sd.lz1 - sd.lz0)));
    }
    const int n = sd.next, ex = sd.ex, ey = sd.ey;
    // LDS: rv[n + 1] (slot n takes the stores of masked steps), cf[n * CS],
    // id[n], each with PAD guard cells on both sides for the padded steps
    // at either end of a sweep
    const RowsLds L = rows_lds(sizeof(VT), sizeof(FT), sizeof(DT), CS, PAD, n);
    VT *rv = reinterpret_cast<VT *>(smem + L.rv) + PAD;
    FT *cf = reinterpret_cast<FT *>(smem + L.cf) + (size_t)PAD * CS;
    static_assert(sizeof(FT) * row_run<BOX, FT>() % 16 == 0, "cell runs are whole 16-byte words");
    DT *id = reinterpret_cast<DT *>(smem + L.id) + PAD;
    const FT *F = reinterpret_cast<const FT *>(a.F);
    const DT *ID = reinterpret_cast<const DT *>(a.invd);
    const size_t fo = sd.fac_off;
    const float inv_ex = 1.0f / (float)ex;
    const int wid = threadIdx.x >> 6;
    // stage: lower runs and R_i^delta r (all threads).  Absent slots and the
    // padding load a valid address and store zero; every load of a pass is
    // issued before its first LDS store.
    for (int c0 = threadIdx.x; c0 < n; c0 += CPT * NT) {
        FT v[CPT][NST];
        double rr[CPT];
        DT dd[CPT];
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = min(c0 + u * NT, n - 1);
#pragma unroll
            for (int q = 0; q < NST; ++q) {
                const int k = a.kmap[q];
                const FT x = F[(size_t)max(k, 0) * a.NE + fo + c];
                v[u][q] = k >= 0 ? x : (FT)0;
            }
            if (ONE) dd[u] = ID[fo + c];
            const int y = row_of(c, inv_ex), x = c - y * ex;
            rr[u] = a.r[(size_t)sd.gorg + x + (size_t)sd.gnx * y];
        }
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = c0 + u * NT;
            if (c < n) {
#pragma unroll
                for (int q = 0; q < NST; ++q) cf[(size_t)c * CS + q] = v[u][q];
                if (ONE) id[c] = dd[u];
                const int y = row_of(c, inv_ex), x = c - y * ex;
                const bool own = x >= sd.lx0 && x < sd.lx1 && y >= sd.ly0 && y < sd.ly1;
                rv[c] = (VT)((a.variant == NKS_RIGHT_RAS && !own) ? 0.0 : rr[u]);
            }
        }
    }
    __syncthreads();
    // one wavefront sweeps, lane = row.  Lanes past the box's rows stay
    // disabled: they take no LDS traffic (a 12-row box leaves 52 of 64 lanes
    // idle), and a lane shift that reads them returns zero, the value of a
    // row outside the box, also through the two-row shifts of the box
    // stencils.
    const int T = (ex - 1) + LB * (ey - 1) + 1;
    const int y = threadIdx.x;
    const bool rowok = y < ey;
    const int ye = min(y, ey - 1);
    const int tlo = rowok ? LB * y : (1 << 28);   // steps with x = t - LB*y inside the row
    const int cb = ye * (ex - LB);                // cell of step t: cb + t (forward)
    // Blocks of RB steps, software pipelined: the LDS reads of the next
    // block are issued before the arithmetic of the current one.  The reads
    // may run ahead of the current block's stores because an active step
    // reads only its own cell, which no other step writes.
    constexpr int RB = RU / 2;
    if (wid == 0 && rowok) {
        // rings: own outputs, outputs of lane y-1 and y-2
        VT r0[RU], r1[RU], r2[RU];
#pragma unroll
        for (int k = 0; k < RU; ++k) r0[k] = r1[k] = r2[k] = (VT)0;
        VT coA[RB][NLP], rinA[RB], coB[RB][NLP], rinB[RB];
        int ccA[RB], ccB[RB];
        bool aaA[RB], aaB[RB];
        auto load = [&](int tb, VT(&co)[RB][NLP], VT(&rin)[RB], int(&cc)[RB], bool(&aa)[RB]) {
            // cells cb + tb + u: within the guard cells for every padded step
            const FT *cfb = cf + (ptrdiff_t)(cb + tb) * CS;
            const VT *rvb = rv + (cb + tb);
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                aa[u] = (unsigned)(tb + u - tlo) < (unsigned)ex;
                cc[u] = cb + tb + u;
                load_run<FT, VT, NLP>(cfb + u * CS, co[u]);
                rin[u] = rvb[u];
            }
        };
        // forward: y_i = r_i - sum_{lower} L_ik y_k.  The terms on outputs at
        // least two steps old do not wait for the previous step: the next
        // step's are summed while this step's dependent chain runs.
        auto older = [&](int uu, const VT(&co)[NLP], VT rin) {
            VT v = rin;
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int h = -(S::DX[q] + LB * S::DY[q]) - 1;
                if (h == 0) continue;
                const int slot = (uu - 1 - h + 2 * RU) % RU;
                const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == -1 ? r1[slot] : r2[slot]);
                v -= co[q] * val;
            }
            return v;
        };
        auto step = [&](int b0, VT(&co)[RB][NLP], VT(&rin)[RB], int(&cc)[RB], bool(&aa)[RB]) {
            VT outv[RB], old[RB];
            old[0] = older(b0, co[0], rin[0]);
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int uu = b0 + u;
                if (u + 1 < RB) old[u + 1] = older(uu + 1, co[u + 1], rin[u + 1]);
                VT v = old[u];
                // the one-step-old terms of this lane, then those that wait
                // for a lane shift (the critical path)
#pragma unroll
                for (int pass = 1; pass < 3; ++pass) {
#pragma unroll
                    for (int q = 0; q < NL; ++q) {
                        const int h = -(S::DX[q] + LB * S::DY[q]) - 1;
                        if (pass != (h != 0 ? 0 : (S::DY[q] == 0 ? 1 : 2))) continue;
                        const int slot = (uu - 1 - h + 2 * RU) % RU;
                        const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == -1 ? r1[slot] : r2[slot]);
                        v -= co[u][q] * val;
                    }
                }
                const VT out = aa[u] ? v : (VT)0;
                outv[u] = out;
                r0[uu] = out;
                r1[uu] = lane_shr(out);
                r2[uu] = lane_shr(r1[uu]);
            }
#pragma unroll
            for (int u = 0; u < RB; ++u) rv[aa[u] ? cc[u] : n] = outv[u];
        };
        // the scheduling barriers keep each block's reads ahead of the
        // previous block's arithmetic (the scheduler would otherwise sink
        // them next to their first use)
        load(0, coA, rinA, ccA, aaA);
        for (int t0 = 0; t0 < T; t0 += RU) {
            load(t0 + RB, coB, rinB, ccB, aaB);
            __builtin_amdgcn_sched_barrier(0);
            step(0, coA, rinA, ccA, aaA);
            load(t0 + RU, coA, rinA, ccA, aaA);
            __builtin_amdgcn_sched_barrier(0);
            step(RB, coB, rinB, ccB, aaB);
        }
    } else if (wid > 0) {
        // the other wavefronts stage the upper runs and 1/u_ii meanwhile
        for (int c0 = threadIdx.x - 64; c0 < n; c0 += CPU * 192) {
            FT v[CPU][NUP];
            DT d[CPU];
#pragma unroll
            for (int u = 0; u < CPU; ++u) {
                const int c = min(c0 + u * 192, n - 1);
#pragma unroll
                for (int q = 0; q < NUP; ++q) {
                    const int k = a.kmap[NLP + q];
                    const FT x = F[(size_t)max(k, 0) * a.NE + fo + c];
                    v[u][q] = k >= 0 ? x : (FT)0;
                }
                d[u] = ID[fo + c];
            }
#pragma unroll
            for (int u = 0; u < CPU; ++u) {
                const int c = c0 + u * 192;
                if (c < n) {
#pragma unroll
                    for (int q = 0; q < NUP; ++q) cf[(size_t)c * CS + NLP + q] = v[u][q];
                    id[c] = d[u];
                }
            }
        }
    }
    __syncthreads();
    if (ONE) {
        // the upper runs over the lower ones, now that the forward sweep is done
        for (int c0 = threadIdx.x; c0 < n; c0 += CPT * NT) {
            FT v[CPT][NUP];
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = min(c0 + u * NT, n - 1);
#pragma unroll
                for (int q = 0; q < NUP; ++q) {
                    const int k = a.kmap[NLP + q];
                    const FT x = F[(size_t)max(k, 0) * a.NE + fo + c];
                    v[u][q] = k >= 0 ? x : (FT)0;
                }
            }
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = c0 + u * NT;
                if (c < n) {
#pragma unroll
                    for (int q = 0; q < NUP; ++q) cf[(size_t)c * CS + q] = v[u][q];
                }
            }
        }
        __syncthreads();
    }
    if (wid == 0 && rowok) {
        // backward: z_i = (y_i - sum_{upper} U_ik z_k) / u_ii, step t at cell cb + (T - 1 - t)
        VT r0[RU], r1[RU], r2[RU];
#pragma unroll
        for (int k = 0; k < RU; ++k) r0[k] = r1[k] = r2[k] = (VT)0;
        const int cbb = cb + T - 1;
        const int tlob = rowok ? T - LB * y - ex : (1 << 28);   // x = T - 1 - t - LB*y in [0, ex)
        VT coA[RB][NUP], rinA[RB], dgA[RB], coB[RB][NUP], rinB[RB], dgB[RB];
        int ccA[RB], ccB[RB];
        bool aaA[RB], aaB[RB];
        auto load = [&](int tb, VT(&co)[RB][NUP], VT(&rin)[RB], VT(&dg)[RB], int(&cc)[RB], bool(&aa)[RB]) {
            // cells cbb - tb - u, addressed from the block's lowest cell
            const int cl = cbb - tb - (RB - 1);
            const FT *cfb = cf + (ptrdiff_t)cl * CS + UOFF;
            const VT *rvb = rv + cl;
            const DT *idb = id + cl;
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                aa[u] = (unsigned)(tb + u - tlob) < (unsigned)ex;
                cc[u] = cl + (RB - 1 - u);
                load_run<FT, VT, NUP>(cfb + (RB - 1 - u) * CS, co[u]);
                rin[u] = rvb[RB - 1 - u];
                dg[u] = (VT)idb[RB - 1 - u];
            }
        };
        auto older = [&](int uu, const VT(&co)[NUP], VT rin) {
            VT v = rin;
#pragma unroll
            for (int q = NL; q < NS; ++q) {
                const int h = S::DX[q] + LB * S::DY[q] - 1;
                if (h == 0) continue;
                const int slot = (uu - 1 - h + 2 * RU) % RU;
                const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == 1 ? r1[slot] : r2[slot]);
                v -= co[q - NL] * val;
            }
            return v;
        };
        auto step = [&](int b0, VT(&co)[RB][NUP], VT(&rin)[RB], VT(&dg)[RB], int(&cc)[RB], bool(&aa)[RB]) {
            VT outv[RB], old[RB];
            old[0] = older(b0, co[0], rin[0]);
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int uu = b0 + u;
                if (u + 1 < RB) old[u + 1] = older(uu + 1, co[u + 1], rin[u + 1]);
                VT v = old[u];
#pragma unroll
                for (int pass = 1; pass < 3; ++pass) {
#pragma unroll
                    for (int q = NL; q < NS; ++q) {
                        const int h = S::DX[q] + LB * S::DY[q] - 1;
                        if (pass != (h != 0 ? 0 : (S::DY[q] == 0 ? 1 : 2))) continue;
                        const int slot = (uu - 1 - h + 2 * RU) % RU;
                        const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == 1 ? r1[slot] : r2[slot]);
                        v -= co[u][q - NL] * val;
                    }
                }
                const VT out = aa[u] ? v * dg[u] : (VT)0;
                outv[u] = out;
                r0[uu] = out;
                r1[uu] = lane_shl(out);
                r2[uu] = lane_shl(r1[uu]);
            }
#pragma unroll
            for (int u = 0; u < RB; ++u) rv[aa[u] ? cc[u] : n] = outv[u];
        };
        load(0, coA, rinA, dgA, ccA, aaA);
        for (int t0 = 0; t0 < T; t0 += RU) {
            load(t0 + RB, coB, rinB, dgB, ccB, aaB);
            __builtin_amdgcn_sched_barrier(0);
            step(0, coA, rinA, dgA, ccA, aaA);
            load(t0 + RU, coA, rinA, dgA, ccA, aaA);
            __builtin_amdgcn_sched_barrier(0);
            step(RB, coB, rinB, dgB, ccB, aaB);
        }
    }
    __syncthreads();
    // write back with all threads, x-contiguous (coalesced)
    if (a.variant == NKS_LEFT_RAS) {
        // WB cells per thread per pass: with accumulation, every load of z
        // is issued before the first store
        constexpr int WB = 4;
        const int oxn = sd.lx1 - sd.lx0, no = oxn * (sd.ly1 - sd.ly0);
        const float inv_oxn = 1.0f / (float)oxn;
        for (int k0 = threadIdx.x; k0 < no; k0 += WB * NT) {
            size_t g[WB];
            double v[WB];
#pragma unroll
            for (int u = 0; u < WB; ++u) {
                const int k = min(k0 + u * NT, no - 1);
                const int yy = row_of(k, inv_oxn), xx = k - yy * oxn;
                const int x = sd.lx0 + xx, yb = sd.ly0 + yy;
                g[u] = (size_t)sd.gorg + x + (size_t)sd.gnx * yb;
                v[u] = (double)rv[yb * ex + x];
            }
            if (a.accumulate) {
#pragma unroll
                for (int u = 0; u < WB; ++u) v[u] += a.z[g[u]];
            }
#pragma unroll
            for (int u = 0; u < WB; ++u)
                if (k0 + u * NT < no) a.z[g[u]] = v[u];
        }
    } else {
        for (int c = threadIdx.x; c < n; c += blockDim.x) a.zext[fo + c] = (double)rv[c];
    }
}

// ---------------------------------------------------------------- kernel: persistent coarse solve
// The coarsest level's GMRES (right-preconditioned by the level's one-level
// left-RAS, restarted every m iterations, one Gram-Schmidt pass, stopped at
// rtol ||b|| or maxit iterations; Remark 2) for every reservoir at once, one
// workgroup per reservoir, with the whole iteration on the device: the
// convergence tests are workgroup-uniform branches, so no host round trip
// and no launch separates two iterations.  The Krylov basis lives in global
// memory (cached); z = M^{-1} v, w = A z and the boxes' extended values in
// LDS.

// One wavefront sweeps a group of boxes packed into its lanes: lane l holds
// row y of one box (the rows of a box on consecutive lanes).  Step t of the
// forward sweep handles x = t - LB*y in every row, the schedule of the
// one-box row sweep; a row's lower neighbours come from its own earlier
// steps and, through the wavefront shifts, from the two rows below.  Every
// shift runs with all lanes of the wavefront enabled, and values cross from
// one box to the next unmasked: a box's factors towards rows outside it are
// exact zeros (those couplings are not in A_i) and every shifted value is
// finite (masked steps give zero), so a neighbouring box's rows contribute
// nothing.  The group runs for its longest box.  The terms of a step on
// outputs at least two steps old are summed for the next step while the
// current step's dependent chain runs.
// Factors are read from per-cell runs in global memory (lower run, then
// upper run), RB steps ahead of the arithmetic; steps outside a row's range
// read a cell clamped into the box and are masked.  Lanes without a row
// (y < 0) compute nothing visible.
// Forward and backward halves of the packed sweep.  The cell runs are read
// from Fb at a stride of CS FT values (0: the lower and upper runs back to
// back), the upper run at offset UOFF (-1: after the lower run), so the same
// code reads per-cell runs in global memory or runs staged in LDS.
template <typename FT, typename VT, typename DT, int BOX, int RB, int CS = 0, int UOFF = -1>
__device__ __forceinline__ void packed_forward(const SubDev &sd, int y, int T, VT *rb, VT *spare, const FT *Fb) {
    using S = RowStencil<BOX>;
    constexpr int NS = S::NS, NL = S::NL, NU = NS - NL, LB = S::LB;
    constexpr int PER = (int)(16 / sizeof(FT));
    constexpr int NLP = row_lpad<BOX, FT>(), NUP = row_upad<BOX, FT>();
    constexpr int RUN = CS > 0 ? CS : row_run<BOX, FT>();   // stride of a cell's runs
    constexpr int UP = UOFF >= 0 ? UOFF : NLP;     // offset of the upper run
    constexpr int RU = rows_unroll(BOX), NB = RU / RB;
    static_assert(NB % 2 == 0 && NB * RB == RU, "an even number of prefetch blocks per ring cycle");
    const bool on = y >= 0;
    const int ex = sd.ex, ey = sd.ey, n = sd.next;
    const int ye = on ? y : 0;
    const int Ts = (ex - 1) + LB * (ey - 1) + 1;
    const int cb = ye * (ex - LB);
    {
        const int tlo = on ? LB * ye : (1 << 28);
        VT r0[RU], r1[RU], r2[RU];
#pragma unroll
        for (int k = 0; k < RU; ++k) r0[k] = r1[k] = r2[k] = (VT)0;
        VT coA[RB][NLP], rinA[RB], coB[RB][NLP], rinB[RB];
        int ccA[RB], ccB[RB];
        bool aaA[RB], aaB[RB];
        auto load = [&](int tb, VT(&co)[RB][NLP], VT(&rin)[RB], int(&cc)[RB], bool(&aa)[RB]) {
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int c = min(max(cb + tb + u, 0), n - 1);
                aa[u] = (unsigned)(tb + u - tlo) < (unsigned)ex;
                cc[u] = c;
                load_run<FT, VT, NLP>(Fb + (size_t)c * RUN, co[u]);
                rin[u] = rb[c];
            }
        };
        // the terms on outputs at least two steps old, summed for the next
        // step while this step's dependent chain runs
        auto older = [&](int uu, const VT(&co)[NLP], VT rin) {
            VT v = rin;
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int h = -(S::DX[q] + LB * S::DY[q]) - 1;
                if (h == 0) continue;
                const int slot = (uu - 1 - h + 2 * RU) % RU;
                const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == -1 ? r1[slot] : r2[slot]);
                v -= co[q] * val;
            }
            return v;
        };
        auto step = [&](int b0, VT(&co)[RB][NLP], VT(&rin)[RB], int(&cc)[RB], bool(&aa)[RB]) {
            VT outv[RB], old[RB];
            old[0] = older(b0, co[0], rin[0]);
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int uu = b0 + u;
                if (u + 1 < RB) old[u + 1] = older(uu + 1, co[u + 1], rin[u + 1]);
                VT v = old[u];
#pragma unroll
                for (int pass = 1; pass < 3; ++pass) {
#pragma unroll
                    for (int q = 0; q < NL; ++q) {
                        const int h = -(S::DX[q] + LB * S::DY[q]) - 1;
                        if (pass != (h != 0 ? 0 : (S::DY[q] == 0 ? 1 : 2))) continue;
                        const int slot = (uu - 1 - h + 2 * RU) % RU;
                        const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == -1 ? r1[slot] : r2[slot]);
                        v -= co[u][q] * val;
                    }
                }
                const VT out = aa[u] ? v : (VT)0;
                outv[u] = out;
                r0[uu] = out;
                r1[uu] = lane_shr(out);
                r2[uu] = lane_shr(r1[uu]);
            }
#pragma unroll
            for (int u = 0; u < RB; ++u) *(aa[u] ? rb + cc[u] : spare) = outv[u];
        };
        load(0, coA, rinA, ccA, aaA);
        for (int t0 = 0; t0 < T; t0 += RU) {
#pragma unroll
            for (int q = 0; q < NB; q += 2) {
                load(t0 + (q + 1) * RB, coB, rinB, ccB, aaB);
                __builtin_amdgcn_sched_barrier(0);
                step(q * RB, coA, rinA, ccA, aaA);
                load(t0 + (q + 2) * RB, coA, rinA, ccA, aaA);
                __builtin_amdgcn_sched_barrier(0);
                step((q + 1) * RB, coB, rinB, ccB, aaB);
            }
        }
    }
}

template <typename FT, typename VT, typename DT, int BOX, int RB, int CS = 0, int UOFF = -1>
__device__ __forceinline__ void packed_backward(const SubDev &sd, int y, int T, VT *rb, VT *spare, const FT *Fb,
                                                const DT *Ib) {
    using S = RowStencil<BOX>;
    constexpr int NS = S::NS, NL = S::NL, NU = NS - NL, LB = S::LB;
    constexpr int PER = (int)(16 / sizeof(FT));
    constexpr int NLP = row_lpad<BOX, FT>(), NUP = row_upad<BOX, FT>();
    constexpr int RUN = CS > 0 ? CS : row_run<BOX, FT>();   // stride of a cell's runs
    constexpr int UP = UOFF >= 0 ? UOFF : NLP;     // offset of the upper run
    constexpr int RU = rows_unroll(BOX), NB = RU / RB;
    static_assert(NB % 2 == 0 && NB * RB == RU, "an even number of prefetch blocks per ring cycle");
    const bool on = y >= 0;
    const int ex = sd.ex, ey = sd.ey, n = sd.next;
    const int ye = on ? y : 0;
    const int Ts = (ex - 1) + LB * (ey - 1) + 1;
    const int cb = ye * (ex - LB);
    {
        // backward: x = Ts - 1 - t - LB*y, upper neighbours from the rows above
        const int cbb = cb + Ts - 1;
        const int tlob = on ? Ts - LB * ye - ex : (1 << 28);
        VT r0[RU], r1[RU], r2[RU];
#pragma unroll
        for (int k = 0; k < RU; ++k) r0[k] = r1[k] = r2[k] = (VT)0;
        VT coA[RB][NUP], rinA[RB], dgA[RB], coB[RB][NUP], rinB[RB], dgB[RB];
        int ccA[RB], ccB[RB];
        bool aaA[RB], aaB[RB];
        auto load = [&](int tb, VT(&co)[RB][NUP], VT(&rin)[RB], VT(&dg)[RB], int(&cc)[RB], bool(&aa)[RB]) {
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int c = min(max(cbb - tb - u, 0), n - 1);
                aa[u] = (unsigned)(tb + u - tlob) < (unsigned)ex;
                cc[u] = c;
                load_run<FT, VT, NUP>(Fb + (size_t)c * RUN + UP, co[u]);
                rin[u] = rb[c];
                dg[u] = (VT)Ib[c];
            }
        };
        auto older = [&](int uu, const VT(&co)[NUP], VT rin) {
            VT v = rin;
#pragma unroll
            for (int q = NL; q < NS; ++q) {
                const int h = S::DX[q] + LB * S::DY[q] - 1;
                if (h == 0) continue;
                const int slot = (uu - 1 - h + 2 * RU) % RU;
                const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == 1 ? r1[slot] : r2[slot]);
                v -= co[q - NL] * val;
            }
            return v;
        };
        auto step = [&](int b0, VT(&co)[RB][NUP], VT(&rin)[RB], VT(&dg)[RB], int(&cc)[RB], bool(&aa)[RB]) {
            VT outv[RB], old[RB];
            old[0] = older(b0, co[0], rin[0]);
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int uu = b0 + u;
                if (u + 1 < RB) old[u + 1] = older(uu + 1, co[u + 1], rin[u + 1]);
                VT v = old[u];
#pragma unroll
                for (int pass = 1; pass < 3; ++pass) {
#pragma unroll
                    for (int q = NL; q < NS; ++q) {
                        const int h = S::DX[q] + LB * S::DY[q] - 1;
                        if (pass != (h != 0 ? 0 : (S::DY[q] == 0 ? 1 : 2))) continue;
                        const int slot = (uu - 1 - h + 2 * RU) % RU;
                        const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == 1 ? r1[slot] : r2[slot]);
                        v -= co[u][q - NL] * val;
                    }
                }
                const VT out = aa[u] ? v * dg[u] : (VT)0;
                outv[u] = out;
                r0[uu] = out;
                r1[uu] = lane_shl(out);
                r2[uu] = lane_shl(r1[uu]);
            }
#pragma unroll
            for (int u = 0; u < RB; ++u) *(aa[u] ? rb + cc[u] : spare) = outv[u];
        };
        load(0, coA, rinA, dgA, ccA, aaA);
        for (int t0 = 0; t0 < T; t0 += RU) {
#pragma unroll
            for (int q = 0; q < NB; q += 2) {
                load(t0 + (q + 1) * RB, coB, rinB, dgB, ccB, aaB);
                __builtin_amdgcn_sched_barrier(0);
                step(q * RB, coA, rinA, dgA, ccA, aaA);
                load(t0 + (q + 2) * RB, coA, rinA, dgA, ccA, aaA);
                __builtin_amdgcn_sched_barrier(0);
                step((q + 1) * RB, coB, rinB, dgB, ccB, aaB);
            }
        }
    }
}

template <typename FT, typename VT, typename DT, int BOX, int RB>
__device__ __forceinline__ void packed_sweep(const SubDev &sd, int y, int T, VT *rb, VT *spare, const FT *Fb,
                                             const DT *Ib) {
    packed_forward<FT, VT, DT, BOX, RB>(sd, y, T, rb, spare, Fb);
    packed_backward<FT, VT, DT, BOX, RB>(sd, y, T, rb, spare, Fb, Ib);
}

// ---------------------------------------------------------------- kernel: packed 2D sweep
// Launches of small boxes (a coarse level's boxes are a dozen rows tall, a
// wavefront sweeping one of them leaves most lanes idle): a workgroup takes
// a group of boxes of one reservoir packed into 64 lanes, the rows of each
// box on consecutive lanes, swept on the schedule of the one-box sweep (see
// packed_forward).  All four wavefronts stage the lower runs and R_i^delta r;
// the first sweeps forward while the others stage the upper runs and
// 1/u_ii; it sweeps back; all write back.  The group's extended cells are
// contiguous in the factor storage, and a per-cell map gives each one's
// global cell (the high bit marks the cells the box owns).
struct PackArgs {
    const SubDev *sub;
    const int2 *glane;      // per group: 64 lanes of {box, row} (row -1: idle)
    const int *gsteps;      // per group: the steps of its longest box
    const int *gbox;        // per group: first box (G + 1 entries)
    const int *ext2glob;    // per extended cell: global cell, high bit set where owned
    const void *F;          // K*NE off-diagonal factors (FT), lexicographic per subdomain
    const void *invd;       // NE (DT)
    int NE;
    const double *r;
    double *z, *zext;
    const int *mask;
    unsigned long long *units;   // profiled launches: swept extended / owned cells
    int variant, accumulate;
    int kmap[32];
};

// LDS of a packed group of n extended cells: rv[n + 1], runs[n * cs], id[n],
// each with guard cells on both sides for the blocks of steps that straddle
// the group's first or last cell
__host__ __device__ constexpr int packed_pad(int box) { return rows_unroll(box) / 2; }
__host__ __device__ inline RowsLds packed_lds(size_t vt, size_t ft, size_t dt, int cs, int box, size_t n) {
    return rows_lds(vt, ft, dt, cs, packed_pad(box), n);
}

// The packed sweeps on LDS-resident runs.  Lane (box, row y) steps through
// the group's cells cg + t (forward; cg = the box's first cell in the group
// plus y (ex - LB)) or cgb - t (backward).  A block of RB steps is addressed
// from one base cell, clamped into the guard cells when the whole block lies
// outside the group (then none of its steps is active), so every load and
// store of a step takes a constant offset from that base; masked steps
// store into the guard cells past the group's end, which no active step
// reads.  Unlike packed_forward / packed_backward, values cross from one box
// to the next through the lane shifts unmasked: a box's factors towards
// rows outside it are exact zeros (those couplings are not in A_i) and every
// shifted value is finite (masked steps give zero), so the neighbouring
// box's rows contribute nothing.
template <typename FT, typename VT, typename DT, int BOX, int RB, int CS, int UP>
__device__ __forceinline__ void lds_forward(int n, int cg, int tlo, int ex, int T, VT *rv, const FT *cf) {
    using S = RowStencil<BOX>;
    constexpr int NL = S::NL, LB = S::LB;
    constexpr int NLP = row_lpad<BOX, FT>();
    constexpr int RU = rows_unroll(BOX), NB = RU / RB;
    static_assert(NB % 2 == 0 && NB * RB == RU, "an even number of prefetch blocks per ring cycle");
    VT *const dum = rv + n;
    VT r0[RU], r1[RU], r2[RU];
#pragma unroll
    for (int k = 0; k < RU; ++k) r0[k] = r1[k] = r2[k] = (VT)0;
    VT coA[RB][NLP], rinA[RB], coB[RB][NLP], rinB[RB];
    int cbA, cbB;
    bool aaA[RB], aaB[RB];
    // run addresses from the first guard cell: a non-negative 24-bit product
    const FT *const cfg = cf - RB * CS;
    auto load = [&](int tb, VT(&co)[RB][NLP], VT(&rin)[RB], int &cb0, bool(&aa)[RB]) {
        cb0 = min(max(cg + tb, -RB), n);
        const FT *cfb = cfg + __umul24((unsigned)(cb0 + RB), (unsigned)CS);
        const VT *rvb = rv + cb0;
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            aa[u] = (unsigned)(tb + u - tlo) < (unsigned)ex;
            load_run<FT, VT, NLP>(cfb + u * CS, co[u]);
            rin[u] = rvb[u];
        }
    };
    // the terms of step u on outputs at least two steps old (available
    // before step u - 1 ends), subtracted from R_i^delta r
    auto older = [&](int uu, const VT(&co)[NLP], VT rin) {
        VT v = rin;
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int h = -(S::DX[q] + LB * S::DY[q]) - 1;
            if (h == 0) continue;
            const int slot = (uu - 1 - h + 2 * RU) % RU;
            const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == -1 ? r1[slot] : r2[slot]);
            v -= co[q] * val;
        }
        return v;
    };
    auto step = [&](int b0, VT(&co)[RB][NLP], VT(&rin)[RB], int cb0, bool(&aa)[RB]) {
        VT outv[RB], old[RB];
        old[0] = older(b0, co[0], rin[0]);
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int uu = b0 + u;
            // the next step's older terms are independent of this step: the
            // two chains interleave
            if (u + 1 < RB) old[u + 1] = older(uu + 1, co[u + 1], rin[u + 1]);
            VT v = old[u];
#pragma unroll
            for (int pass = 1; pass < 3; ++pass) {
#pragma unroll
                for (int q = 0; q < NL; ++q) {
                    const int h = -(S::DX[q] + LB * S::DY[q]) - 1;
                    if (pass != (h != 0 ? 0 : (S::DY[q] == 0 ? 1 : 2))) continue;
                    const int slot = (uu - 1 - h + 2 * RU) % RU;
                    const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == -1 ? r1[slot] : r2[slot]);
                    v -= co[u][q] * val;
                }
            }
            const VT out = aa[u] ? v : (VT)0;
            outv[u] = out;
            r0[uu] = out;
            r1[uu] = lane_shr(out);
            r2[uu] = lane_shr(r1[uu]);
        }
        VT *const rvb = rv + cb0;
#pragma unroll
        for (int u = 0; u < RB; ++u) (aa[u] ? rvb : dum)[u] = outv[u];
    };
    load(0, coA, rinA, cbA, aaA);
    for (int t0 = 0; t0 < T; t0 += RU) {
#pragma unroll
        for (int q = 0; q < NB; q += 2) {
            load(t0 + (q + 1) * RB, coB, rinB, cbB, aaB);
            __builtin_amdgcn_sched_barrier(0);
            step(q * RB, coA, rinA, cbA, aaA);
            load(t0 + (q + 2) * RB, coA, rinA, cbA, aaA);
            __builtin_amdgcn_sched_barrier(0);
            step((q + 1) * RB, coB, rinB, cbB, aaB);
        }
    }
}

template <typename FT, typename VT, typename DT, int BOX, int RB, int CS, int UP>
__device__ __forceinline__ void lds_backward(int n, int cgb, int tlob, int ex, int T, VT *rv, const FT *cf,
                                             const DT *id) {
    using S = RowStencil<BOX>;
    constexpr int NS = S::NS, NL = S::NL, LB = S::LB;
    constexpr int NUP = row_upad<BOX, FT>();
    constexpr int RU = rows_unroll(BOX), NB = RU / RB;
    static_assert(NB % 2 == 0 && NB * RB == RU, "an even number of prefetch blocks per ring cycle");
    VT *const dum = rv + n;
    VT r0[RU], r1[RU], r2[RU];
#pragma unroll
    for (int k = 0; k < RU; ++k) r0[k] = r1[k] = r2[k] = (VT)0;
    VT coA[RB][NUP], rinA[RB], dgA[RB], coB[RB][NUP], rinB[RB], dgB[RB];
    int clA, clB;
    bool aaA[RB], aaB[RB];
    // block of steps tb .. tb + RB - 1 at cells cgb - tb - u, addressed from
    // its lowest cell
    const FT *const cfg = cf - RB * CS + UP;
    auto load = [&](int tb, VT(&co)[RB][NUP], VT(&rin)[RB], VT(&dg)[RB], int &cl, bool(&aa)[RB]) {
        cl = min(max(cgb - tb - (RB - 1), -RB), n);
        const FT *cfb = cfg + __umul24((unsigned)(cl + RB), (unsigned)CS);
        const VT *rvb = rv + cl;
        const DT *idb = id + cl;
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            aa[u] = (unsigned)(tb + u - tlob) < (unsigned)ex;
            load_run<FT, VT, NUP>(cfb + (RB - 1 - u) * CS, co[u]);
            rin[u] = rvb[RB - 1 - u];
            dg[u] = (VT)idb[RB - 1 - u];
        }
    };
    auto older = [&](int uu, const VT(&co)[NUP], VT rin) {
        VT v = rin;
#pragma unroll
        for (int q = NL; q < NS; ++q) {
            const int h = S::DX[q] + LB * S::DY[q] - 1;
            if (h == 0) continue;
            const int slot = (uu - 1 - h + 2 * RU) % RU;
            const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == 1 ? r1[slot] : r2[slot]);
            v -= co[q - NL] * val;
        }
        return v;
    };
    auto step = [&](int b0, VT(&co)[RB][NUP], VT(&rin)[RB], VT(&dg)[RB], int cl, bool(&aa)[RB]) {
        VT outv[RB], old[RB];
        old[0] = older(b0, co[0], rin[0]);
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int uu = b0 + u;
            if (u + 1 < RB) old[u + 1] = older(uu + 1, co[u + 1], rin[u + 1]);
            VT v = old[u];
#pragma unroll
            for (int pass = 1; pass < 3; ++pass) {
#pragma unroll
                for (int q = NL; q < NS; ++q) {
                    const int h = S::DX[q] + LB * S::DY[q] - 1;
                    if (pass != (h != 0 ? 0 : (S::DY[q] == 0 ? 1 : 2))) continue;
                    const int slot = (uu - 1 - h + 2 * RU) % RU;
                    const VT val = S::DY[q] == 0 ? r0[slot] : (S::DY[q] == 1 ? r1[slot] : r2[slot]);
                    v -= co[u][q - NL] * val;
                }
            }
            const VT out = aa[u] ? v * dg[u] : (VT)0;
            outv[u] = out;
            r0[uu] = out;
            r1[uu] = lane_shl(out);
            r2[uu] = lane_shl(r1[uu]);
        }
        VT *const rvb = rv + cl;
#pragma unroll
        for (int u = 0; u < RB; ++u) (aa[u] ? rvb : dum)[RB - 1 - u] = outv[u];
    };
    load(0, coA, rinA, dgA, clA, aaA);
    for (int t0 = 0; t0 < T; t0 += RU) {
#pragma unroll
        for (int q = 0; q < NB; q += 2) {
            load(t0 + (q + 1) * RB, coB, rinB, dgB, clB, aaB);
            __builtin_amdgcn_sched_barrier(0);
            step(q * RB, coA, rinA, dgA, clA, aaA);
            load(t0 + (q + 2) * RB, coA, rinA, dgA, clA, aaA);
            __builtin_amdgcn_sched_barrier(0);
            step((q + 1) * RB, coB, rinB, dgB, clB, aaB);
        }
    }
}

template <typename FT, typename VT, typename DT, int BOX>
__global__ void __launch_bounds__(256) k_ras_packed(PackArgs a) {
    using S = RowStencil<BOX>;
    constexpr int NL = S::NL, NU = S::NS - NL;
    constexpr int PER = (int)(16 / sizeof(FT));
    constexpr int NLP = row_lpad<BOX, FT>(), NUP = row_upad<BOX, FT>();
    constexpr int CS = row_stride<BOX, FT>();
    constexpr int RB = rows_unroll(BOX) / 2;
    constexpr int CPT = 2;   // cells per thread per staging pass
    extern __shared__ __align__(16) unsigned char smem[];
    const int g = blockIdx.x, tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const int b0 = a.gbox[g], b1 = a.gbox[g + 1];
    const SubDev first = a.sub[b0];
    if (a.mask && !a.mask[first.blk]) return;
    const SubDev last = a.sub[b1 - 1];
    const int e0 = first.fac_off, n = last.fac_off + last.next - e0;
    constexpr int PAD = packed_pad(BOX);
    const RowsLds L = packed_lds(sizeof(VT), sizeof(FT), sizeof(DT), CS, BOX, n);
    VT *rv = reinterpret_cast<VT *>(smem + L.rv) + PAD;
    FT *cf = reinterpret_cast<FT *>(smem + L.cf) + PAD * CS;
    DT *id = reinterpret_cast<DT *>(smem + L.id) + PAD;
    const FT *F = reinterpret_cast<const FT *>(a.F);
    const DT *ID = reinterpret_cast<const DT *>(a.invd);
    const int *e2g = a.ext2glob + e0;
    // the lower runs and R_i^delta r (right-RAS: zero off the owned cells)
    for (int c0 = tid; c0 < n; c0 += CPT * 256) {
        FT v[CPT][NLP];
        double rr[CPT];
        int gg[CPT];
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = min(c0 + u * 256, n - 1);
#pragma unroll
            for (int q = 0; q < NLP; ++q) {
                const int k = a.kmap[q];
                const FT x = F[(size_t)max(k, 0) * a.NE + e0 + c];
                v[u][q] = k >= 0 ? x : (FT)0;
            }
            gg[u] = e2g[c];
            rr[u] = a.r[gg[u] & 0x7fffffff];
        }
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = c0 + u * 256;
            if (c < n) {
#pragma unroll
                for (int q = 0; q < NLP; ++q) cf[(size_t)c * CS + q] = v[u][q];
                rv[c] = (VT)((a.variant == NKS_RIGHT_RAS && gg[u] >= 0) ? 0.0 : rr[u]);
            }
        }
    }
    __syncthreads();
    const int2 ln = a.glane[(size_t)g * 64 + lane];
    const SubDev sd = a.sub[ln.x];
    const int T = a.gsteps[g];
    // this lane's row: first group cell of its forward and backward steps and
    // the steps at which its row starts
    const bool on = ln.y >= 0;
    const int ye = on ? ln.y : 0, ex = sd.ex, ey = sd.ey;
    const int Ts = (ex - 1) + S::LB * (ey - 1) + 1;
    const int cg = (sd.fac_off - e0) + ye * (ex - S::LB);
    const int tlo = on ? S::LB * ye : (1 << 28), tlob = on ? Ts - S::LB * ye - ex : (1 << 28);
    if (wid == 0) {
        lds_forward<FT, VT, DT, BOX, RB, CS, NLP>(n, cg, tlo, ex, T, rv, cf);
    } else {
        // the upper runs and 1/u_ii meanwhile
        for (int c0 = tid - 64; c0 < n; c0 += CPT * 192) {
            FT v[CPT][NUP];
            DT d[CPT];
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = min(c0 + u * 192, n - 1);
#pragma unroll
                for (int q = 0; q < NUP; ++q) {
                    const int k = a.kmap[NLP + q];
                    const FT x = F[(size_t)max(k, 0) * a.NE + e0 + c];
                    v[u][q] = k >= 0 ? x : (FT)0;
                }
                d[u] = ID[e0 + c];
            }
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = c0 + u * 192;
                if (c < n) {
#pragma unroll
                    for (int q = 0; q < NUP; ++q) cf[(size_t)c * CS + NLP + q] = v[u][q];
                    id[c] = d[u];
                }
            }
        }
    }
    __syncthreads();
    if (wid == 0)
        lds_backward<FT, VT, DT, BOX, RB, CS, NLP>(n, cg + Ts - 1, tlob, ex, T, rv, cf, id);
    __syncthreads();
    // write back: the owned cells (left-RAS), or every extended cell for the gather
    unsigned long long own = 0;
    for (int c = tid; c < n; c += 256) {
        if (a.variant == NKS_LEFT_RAS) {
            const int gg = e2g[c];
            if (gg < 0) {
                const size_t gi = (size_t)(gg & 0x7fffffff);
                const double v = (double)rv[c];
                a.z[gi] = a.accumulate ? a.z[gi] + v : v;
                ++own;
            }
        } else {
            a.zext[e0 + c] = (double)rv[c];
        }
    }
    if (a.units) {
        // spread over PROF_UNIT_SLOTS counter pairs, so the workgroups of a
        // launch do not queue on one address
        unsigned long long *u = a.units + 2 * (blockIdx.x % PROF_UNIT_SLOTS);
        if (tid == 0) atomicAdd(u, (unsigned long long)n);
        if (own) atomicAdd(u + 1, own);
    }
}

constexpr int COARSE_CELLS = 4096;   // cells of a reservoir on the coarsest level, at most
constexpr size_t COARSE_AUTO_RUN_BYTES = 256 * 1024;   // factor runs of a reservoir, automatic choice

struct CoarseArgs {
    const Blk *blk;          // the level's reservoirs (2D)
    const SubDev *sub;       // the level's boxes
    const int *efirst;       // per reservoir: first extended cell (B + 1 entries)
    const int *gfirst;       // per reservoir: first lane group (B + 1 entries)
    const int2 *glane;       // per group: 64 lanes of {box, row} (row -1: idle)
    const int *gsteps;       // per group: the steps of its longest box
    const int *ext2loc;      // per extended cell: the reservoir-local cell it copies
    const int *own2ext;      // per cell: the extended cell of the box that owns it
    const void *runs;        // per extended cell: the padded lower and upper factor runs (FT)
    const void *invd;        // per extended cell: 1/u_ii (DT)
    const double *coef;      // the level's operator, K x N
    int K, N;
    int offp[25];            // the operator's (dx, dy) in the low two bytes
    const double *b;
    double *x;
    double *V;               // basis: reservoir b's m + 1 columns of n_b at V + (m + 1) off_b
    const int *mask;
    int *its;                // per reservoir: iterations taken
    double *res;             // per reservoir: the last residual estimate
    int m, maxit;
    double rtol, atol;
    int ncap;                // cells of the largest reservoir (LDS sizing)
};

// Workgroup sums of eight per-thread columns in a fixed order: within a
// wavefront by recursive halving over the lane bits (after the exchange
// across bit k a lane keeps the half of its columns that bit selects, so
// lane l ends with column (l >> 3) & 7 summed over the wavefront), then the
// wavefront totals in wavefront order into out[0..7].  red holds eight
// doubles per wavefront.  Every thread of the workgroup calls it.
template <int NT>
__device__ __forceinline__ void workgroup_sum8(double (&a)[8], double *red, double *out) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool hi = lane & 32;
        const double keep = hi ? a[k + 4] : a[k], send = hi ? a[k] : a[k + 4];
        a[k] = keep + __shfl_xor(send, 32);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const bool hi = lane & 16;
        const double keep = hi ? a[k + 2] : a[k], send = hi ? a[k] : a[k + 2];
        a[k] = keep + __shfl_xor(send, 16);
    }
    {
        const bool hi = lane & 8;
        const double keep = hi ? a[1] : a[0], send = hi ? a[0] : a[1];
        a[0] = keep + __shfl_xor(send, 8);
    }
    a[0] += __shfl_xor(a[0], 4);
    a[0] += __shfl_xor(a[0], 2);
    a[0] += __shfl_xor(a[0], 1);
    if ((lane & 7) == 0) red[wid * 8 + (lane >> 3)] = a[0];
    __syncthreads();
    if ((int)threadIdx.x < 8) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w * 8 + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// stencil points of the coarse operator per row template (5-point cross,
// 5x5 box, 21-point)
template <int BOX> constexpr int coarse_kmax() { return BOX == 0 ? 5 : (BOX == 1 ? 25 : 21); }

template <typename FT, typename VT, typename DT, int BOX, int NT>
__global__ void __launch_bounds__(NT) k_coarse_gmres(CoarseArgs a) {
    constexpr int NW = NT / 64;
    constexpr int RB = BOX == 0 ? 4 : 2;
    constexpr int CPT = COARSE_CELLS / NT;   // cells per thread at most
    constexpr int KMAX = coarse_kmax<BOX>();
    extern __shared__ __align__(16) unsigned char smem[];
    const int bi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const Blk k = a.blk[bi];
    const int n = k.nx * k.ny, nx = k.nx;
    double *xg = a.x + k.off;
    const double *bg = a.b + k.off;
    if (a.mask && !a.mask[bi]) {
        for (int i = tid; i < n; i += NT) xg[i] = 0.0;
        if (tid == 0) {
            a.its[bi] = 0;
            a.res[bi] = 0.0;
        }
        return;
    }
    const int m = a.m;
    // LDS: z and w (ncap doubles each), column totals, the rotated
    // Hessenberg columns (m x m), rotations, g, y, wavefront partials,
    // flags, extended values
    double *zl = reinterpret_cast<double *>(smem);
    double *wl = zl + a.ncap;
    double *hc = wl + a.ncap;
    double *H = hc + 40;
    double *cs = H + m * m, *sn = cs + m, *g = sn + m, *yv = g + m + 1;
    double *red = yv + m;
    int *flag = reinterpret_cast<int *>(red + 8 * NW);
    VT *rv = reinterpret_cast<VT *>(flag + 4);
    const int e0 = a.efirst[bi], ne = a.efirst[bi + 1] - e0;
    VT *spare = rv + ne;
    const FT *runs = reinterpret_cast<const FT *>(a.runs);
    const DT *ID = reinterpret_cast<const DT *>(a.invd);
    double *Vb = a.V + (size_t)(m + 1) * k.off;
    const int K = a.K;
    const double *coef = a.coef + k.off;
    // dst_i = (A src)_i (minus from b_i when b is given) for the cells of
    // this thread, every coefficient load of a cell issued together; a
    // neighbour outside the reservoir has a zero coefficient, so its index
    // is only clamped
    auto spmv = [&](const double *src, double *dst, const double *bb) {
#pragma unroll 1
        for (int u = 0; u < CPT; ++u) {
            int i = tid + u * NT;
            if (i < n) {
                // the empty asm keeps the address arithmetic here (hoisted out
                // of the solve it would hold a register per point); rows past
                // K load row K - 1 and are dropped by a select, so every load
                // of the cell is issued together
                asm volatile("" : "+v"(i));
                double cv[KMAX];
#pragma unroll
                for (int q = 0; q < KMAX; ++q) cv[q] = coef[(unsigned)(min(q, K - 1) * a.N + i)];
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < KMAX; ++q) {
                    const int o = a.offp[q];
                    const int lq = (int)(int8_t)(o & 0xff) + nx * (int)(int8_t)((o >> 8) & 0xff);
                    const double t = cv[q] * src[(unsigned)min(max(i + lq, 0), n - 1)];
                    s += q < K ? t : 0.0;
                }
                dst[i] = bb ? bb[i] - s : s;
            }
        }
    };
    // zl = M^{-1} src: restricted input on every box, sweeps, owned cells
    auto precondition = [&](const double *src) {
        // four cells per thread per pass: the index loads, then the value loads
        for (int eb = 0; eb < ne; eb += 4 * NT) {
            int ix[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) ix[u] = a.ext2loc[e0 + min(eb + tid + u * NT, ne - 1)];
            double xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = src[ix[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (eb + tid + u * NT < ne) rv[eb + tid + u * NT] = (VT)xv[u];
        }
        __syncthreads();
        for (int q = a.gfirst[bi] + wid; q < a.gfirst[bi + 1]; q += NW) {
            const int2 ln = a.glane[(size_t)q * 64 + lane];
            const SubDev sd = a.sub[ln.x];
            packed_sweep<FT, VT, DT, BOX, RB>(sd, ln.y, a.gsteps[q], rv + (sd.fac_off - e0), spare,
                                              runs + (size_t)sd.fac_off * row_run<BOX, FT>(), ID + sd.fac_off);
        }
        __syncthreads();
        int ox[CPT];
#pragma unroll
        for (int u = 0; u < CPT; ++u) ox[u] = a.own2ext[k.off + min(tid + u * NT, n - 1)];
#pragma unroll
        for (int u = 0; u < CPT; ++u)
            if (tid + u * NT < n) zl[tid + u * NT] = (double)rv[ox[u] - e0];
        __syncthreads();
    };
    // hc[c] = wl . V_c for c < nv, and hc[nv] = wl . wl: eight columns at a
    // time, every load of a thread's cells issued together, fixed-order sums
    auto dots = [&](int nv) {
        for (int c0 = 0; c0 <= nv; c0 += 8) {
            double acc[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[c] = 0.0;
#pragma unroll 1
            for (int u = 0; u < CPT; ++u) {
                int i = tid + u * NT;
                if (i < n) {
                    asm volatile("" : "+v"(i));
                    const double w = wl[i];
                    // columns past the basis load column 0 (allocated, possibly
                    // never written) and are dropped by a select
                    double v[8];
#pragma unroll
                    for (int c = 0; c < 8; ++c) v[c] = Vb[(unsigned)((c0 + c < nv ? c0 + c : 0) * n + i)];
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int cc = c0 + c;
                        acc[c] += cc < nv ? w * v[c] : (cc == nv ? w * w : 0.0);
                    }
                }
            }
            workgroup_sum8<NT>(acc, red, hc + c0);
        }
    };
    // dst_i = scale (base_i - sum_{c < nc} coefs[c] V_c[i]), or
    // scale sum_{c < nc} coefs[c] V_c[i] without a base
    auto combine = [&](const double *base, const double *coefs, int nc, double scale, double *dst) {
#pragma unroll 1
        for (int u = 0; u < CPT; ++u) {
            int i = tid + u * NT;
            if (i < n) {
                asm volatile("" : "+v"(i));
                double t = 0.0;
                for (int c0 = 0; c0 < nc; c0 += 8) {
                    double v[8];
#pragma unroll
                    for (int c = 0; c < 8; ++c) v[c] = Vb[(unsigned)((c0 + c < nc ? c0 + c : 0) * n + i)];
#pragma unroll
                    for (int c = 0; c < 8; ++c) t += c0 + c < nc ? coefs[c0 + c] * v[c] : 0.0;
                }
                dst[i] = (base ? base[i] - t : t) * scale;
            }
        }
    };
    // x = 0, r = b
    for (int i = tid; i < n; i += NT) {
        xg[i] = 0.0;
        wl[i] = bg[i];
    }
    __syncthreads();
    dots(0);
    double beta = sqrt(hc[0]);
    const double tol = fmax(a.rtol * beta, a.atol);
    int its = 0;
    double res = beta;
    for (;;) {
        if (beta <= tol || its >= a.maxit) break;
        const double ib = 1.0 / beta;
        for (int i = tid; i < n; i += NT) Vb[i] = wl[i] * ib;
        if (tid == 0) {
            g[0] = beta;
            for (int j = 1; j <= m; ++j) g[j] = 0.0;
        }
        __syncthreads();
        int kdim = 0, conv = 0;
        for (int j = 0; j < m; ++j) {
            precondition(Vb + (size_t)j * n);
            // w = A z; h = V[0..j]^T w and w.w (one pass)
            spmv(zl, wl, nullptr);
            __syncthreads();
            dots(j + 1);
            double h2 = 0.0;
            for (int c = 0; c <= j; ++c) h2 += hc[c] * hc[c];
            const double hn = sqrt(fmax(hc[j + 1] - h2, 0.0));
            if (hn > 0.0) combine(wl, hc, j + 1, 1.0 / hn, Vb + (size_t)(j + 1) * n);
            if (tid == 0) {
                // column j: h, the earlier rotations, then the new one
                double *col = H + (size_t)j * m;
                for (int c = 0; c <= j; ++c) col[c] = hc[c];
                for (int c = 0; c < j; ++c) {
                    const double a0 = col[c], a1 = col[c + 1];
                    col[c] = cs[c] * a0 + sn[c] * a1;
                    col[c + 1] = -sn[c] * a0 + cs[c] * a1;
                }
                const double a0 = col[j];
                const double den = sqrt(a0 * a0 + hn * hn);
                const double c = den > 0.0 ? a0 / den : 1.0;
                const double s = den > 0.0 ? hn / den : 0.0;
                col[j] = den;
                cs[j] = c;
                sn[j] = s;
                const double gj = g[j];
                g[j + 1] = -s * gj;
                g[j] = c * gj;
                const double r = fabs(s * gj);
                flag[0] = (r <= tol || hn == 0.0) ? 1 : 0;
                hc[39] = r;   // read back after the barrier
            }
            __syncthreads();
            ++its;
            kdim = j + 1;
            conv = flag[0];
            res = hc[39];
            __syncthreads();   // hc and flag are rewritten by the next iteration
            if (conv || its >= a.maxit) break;
        }
        // y = R^{-1} g by columns, then u = V y into column kdim (no longer
        // needed), x += M^{-1} u
        if (tid == 0) {
            for (int c = 0; c < kdim; ++c) yv[c] = g[c];
            for (int c = kdim - 1; c >= 0; --c) {
                const double yc = yv[c] / H[(size_t)c * m + c];
                yv[c] = yc;
                for (int i = 0; i < c; ++i) yv[i] -= H[(size_t)c * m + i] * yc;
            }
        }
        __syncthreads();
        combine(nullptr, yv, kdim, 1.0, Vb + (size_t)kdim * n);
        __syncthreads();
        precondition(Vb + (size_t)kdim * n);
        for (int i = tid; i < n; i += NT) xg[i] += zl[i];
        if (conv || its >= a.maxit) break;
        __syncthreads();
        // restart: r = b - A x
        spmv(xg, wl, bg);
        __syncthreads();
        dots(0);
        beta = sqrt(hc[0]);
        res = beta;
    }
    if (tid == 0) {
        a.its[bi] = its;
        a.res[bi] = res;
    }
}

// per-cell factor runs for the persistent coarse solve: run[e][q] = F[kmap[q]][e]
template <typename FT, int RUN>
__global__ void k_pack_runs(const FT *F, int NE, const int *kmap, FT *runs) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NE) return;
#pragma unroll
    for (int q = 0; q < RUN; ++q) {
        const int k = kmap[q];
        runs[(size_t)e * RUN + q] = k >= 0 ? F[(size_t)k * NE + e] : (FT)0;
    }
}

// ---------------------------------------------------------------- kernel: 3D row sweep
// 3D boxes with the 7-point stencil and rows of at most 64 cells: lane
// r = y + ey*z owns row (y, z) (boxes of more than 64 rows are split into
// slabs of z planes, one wavefront each), and step t handles x = t - y - z, so the
// three lower neighbours of a cell were produced one step earlier: by this
// lane (x-1), by lane r-1 (y-1, through a DPP lane shift) and by lane r-ey
// (z-1, through a lane permute).  Neighbours outside the box have zero
// factors (they are dropped from A_i), so what those lanes hold only has to
// be finite; rows past the box and steps outside a row's range are masked
// to zero.  The backward sweep mirrors this with the upper neighbours.
// Factors, 1/u_ii and R_i^delta r are staged in LDS as in the 2D sweep.
// padded length of a cell's lower (and of its upper) run in the 3D row
// sweep: a whole 16-byte word of FT, or, where both runs of three fit one
// word (BF16), four values each, so a box's runs take 16 B per cell
template <typename FT>
__host__ __device__ constexpr int rows3d_lpad() {
    return 6 * sizeof(FT) <= 16 ? 4 : (3 + (int)(16 / sizeof(FT)) - 1) / (int)(16 / sizeof(FT)) * (int)(16 / sizeof(FT));
}

struct Rows3Args {
    const SubDev *sub;
    const void *F;        // K*NE off-diagonal factors (FT), lexicographic per subdomain
    const void *invd;     // NE (DT)
    int NE;
    const double *r;
    double *z, *zext;
    const int *mask;
    unsigned long long *units;   // profiled launches: swept extended / owned cells
    int *err;             // the level's error word: bit 2 set when a bounded wait gives up
    int variant, accumulate;
    int kmap[16];         // run slot -> stencil index: lower (z, y, x) then upper (x, y, z); -1 padding
};

// HALF: LDS holds one run per cell at a time (boxes whose two runs do not
// fit): the lower runs are staged for the forward sweep, then the upper runs
// and 1/u_ii take their place for the backward sweep.
template <typename FT, typename VT, typename DT, bool MULTI, int NT, bool HALF>
__global__ void __launch_bounds__(NT) k_ras_rows3d(Rows3Args a) {
    constexpr int NLP = rows3d_lpad<FT>();           // lower run: Lz, Ly, Lx, padding
    constexpr int NSP = 2 * NLP;                     // then the upper run: Ux, Uy, Uz, padding
    constexpr int CST = HALF ? NLP : NSP;            // LDS stride of a cell's runs
    constexpr int NST = HALF ? NLP : NSP;            // run slots staged before the forward sweep
    constexpr int NWV = NT / 64;                     // wavefronts: at most this many slabs
    constexpr int RB = MULTI ? 4 : 8;                // steps per block of LDS reads
    constexpr int CPT = 2;
    extern __shared__ __align__(16) unsigned char smem3[];
    __shared__ int prog[2][NWV];                     // steps done per slab: forward, backward
    const SubDev sd = a.sub[blockIdx.x];
    if (a.mask && !a.mask[sd.blk]) return;
    if (a.units && threadIdx.x == 0) {
        // spread over PROF_UNIT_SLOTS counter pairs, so the workgroups of a
        // launch do not queue on one address
        unsigned long long *u = a.units + 2 * (blockIdx.x % PROF_UNIT_SLOTS);
        atomicAdd(u, (unsigned long long)sd.next);
        atomicAdd(u + 1, (unsigned long long)((sd.lx1 - sd.lx0) * (sd.ly1 - sd.ly0) * (sd.lz1 - sd.lz0)));
    }
    const int n = sd.next, ex = sd.ex, ey = sd.ey, ez = sd.ez;
    if (MULTI && threadIdx.x < 2 * NWV) prog[threadIdx.x / NWV][threadIdx.x % NWV] = 0;
    VT *rv = reinterpret_cast<VT *>(smem3);
    FT *cf = reinterpret_cast<FT *>(smem3 + al16(sizeof(VT) * (size_t)(n + 1)));
    DT *id = reinterpret_cast<DT *>(smem3 + al16(sizeof(VT) * (size_t)(n + 1)) + al16(sizeof(FT) * (size_t)CST * n));
    const FT *F = reinterpret_cast<const FT *>(a.F);
    const DT *ID = reinterpret_cast<const DT *>(a.invd);
    const size_t fo = sd.fac_off;
    const float inv_ex = 1.0f / (float)ex, inv_ey = 1.0f / (float)ey;
    // stage every cell's runs, 1/u_ii and R_i^delta r; every load of a pass
    // is issued before its first LDS store
    for (int c0 = threadIdx.x; c0 < n; c0 += CPT * NT) {
        FT v[CPT][NST];
        DT d[CPT];
        double rr[CPT];
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = min(c0 + u * NT, n - 1);
#pragma unroll
            for (int q = 0; q < NST; ++q) {
                const int k = a.kmap[q];
                const FT x = F[(size_t)max(k, 0) * a.NE + fo + c];
                v[u][q] = k >= 0 ? x : (FT)0;
            }
            if (!HALF) d[u] = ID[fo + c];
            const int row = row_of(c, inv_ex), x = c - row * ex;
            const int z = row_of(row, inv_ey), y = row - z * ey;
            rr[u] = a.r[(size_t)sd.gorg + x + (size_t)sd.gnx * (y + (size_t)sd.gny * z)];
        }
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = c0 + u * NT;
            if (c < n) {
#pragma unroll
                for (int q = 0; q < NST; ++q) cf[(size_t)c * CST + q] = v[u][q];
                if (!HALF) id[c] = d[u];
                const int row = row_of(c, inv_ex), x = c - row * ex;
                const int z = row_of(row, inv_ey), y = row - z * ey;
                const bool own = x >= sd.lx0 && x < sd.lx1 && y >= sd.ly0 && y < sd.ly1 && z >= sd.lz0 && z < sd.lz1;
                rv[c] = (VT)((a.variant == NKS_RIGHT_RAS && !own) ? 0.0 : rr[u]);
            }
        }
    }
    __syncthreads();
    // MULTI: the box's z planes are split into slabs of pz planes, one
    // sweeping wavefront each.  A slab's first plane takes its z-1 values
    // from the LDS copy the slab below has written, after waiting for that
    // wavefront's progress counter; the backward sweep mirrors this with the
    // slab above.  Every wait ends: the lowest slab (forward) and the highest
    // (backward) never wait, and a spin limit bounds each wait.
    const int pz = MULTI ? 64 / ey : ez;          // planes per sweeping wavefront
    const int W = MULTI ? (ez + pz - 1) / pz : 1;
    const int w = threadIdx.x >> 6;
    // a wait that reaches the spin limit marks the level's error word, so the
    // next check reports the call as failed instead of returning a sweep over
    // stale values
    auto wait_for = [&](const int *p, int need) {
        int spins = 0;
        while (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < need) {
            if (++spins >= (1 << 22)) {
                if ((threadIdx.x & 63) == 0) atomicOr(a.err, 2);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    };
    const int r = threadIdx.x & 63;
    const int zl = r / ey, y0 = r - zl * ey;
    const int nzw = min(pz, ez - w * pz);        // planes of this slab
    const bool rowok = zl < nzw;
    const int y = rowok ? y0 : 0, z = w * pz + (rowok ? zl : 0);
    const int exy = ex * ey;
    const int T = (ex - 1) + (ey - 1) + (ez - 1) + 1;
    const int lo = rowok ? y + z : (1 << 28);     // steps with x inside the row
    const int cb = ex * (y + ey * z) - y - z;     // cell of forward step t: cb + t
    const int pz_f = ((r - ey) & 63) << 2, pz_b = ((r + ey) & 63) << 2;   // permute sources
    const bool zfirst = MULTI && w > 0 && zl == 0;             // z-1 from the slab below
    const bool zlast = MULTI && w < W - 1 && zl == nzw - 1;    // z+1 from the slab above
    if (w < W) {
        // forward: y_i = r_i - Lz y_(z-1) - Ly y_(y-1) - Lx y_(x-1)
        VT prev = (VT)0;
        for (int t0 = 0; t0 < T; t0 += RB) {
            if (MULTI && w > 0) wait_for(&prog[0][w - 1], min(t0 + RB, T));
            VT co[RB][NLP], rin[RB], rz[RB];
            int cc[RB];
            bool aa[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int t = t0 + u;
                aa[u] = (unsigned)(t - lo) < (unsigned)ex;
                cc[u] = min(max(cb + t, 0), n - 1);
                load_run<FT, VT, NLP>(cf + (size_t)cc[u] * CST, co[u]);
                rin[u] = rv[cc[u]];
                if (MULTI) rz[u] = rv[max(cc[u] - exy, 0)];
            }
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const VT yp = lane_shr(prev);
                VT zp = lane_from(prev, pz_f);
                if (MULTI) zp = zfirst ? rz[u] : zp;
                VT v = rin[u];
                v -= co[u][0] * zp;
                v -= co[u][1] * yp;
                v -= co[u][2] * prev;
                prev = aa[u] ? v : (VT)0;
                rv[aa[u] ? cc[u] : n] = prev;
            }
            if (MULTI) __hip_atomic_store(&prog[0][w], t0 + RB, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    if (HALF) {
        // the upper runs and 1/u_ii over the lower runs
        __syncthreads();
        for (int c0 = threadIdx.x; c0 < n; c0 += CPT * NT) {
            FT v[CPT][NLP];
            DT d[CPT];
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = min(c0 + u * NT, n - 1);
#pragma unroll
                for (int q = 0; q < NLP; ++q) {
                    const int k = a.kmap[NLP + q];
                    const FT x = F[(size_t)max(k, 0) * a.NE + fo + c];
                    v[u][q] = k >= 0 ? x : (FT)0;
                }
                d[u] = ID[fo + c];
            }
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = c0 + u * NT;
                if (c < n) {
#pragma unroll
                    for (int q = 0; q < NLP; ++q) cf[(size_t)c * CST + q] = v[u][q];
                    id[c] = d[u];
                }
            }
        }
        __syncthreads();
    }
    if (w < W) {
        // backward: z_i = (y_i - Ux z_(x+1) - Uy z_(y+1) - Uz z_(z+1)) / u_ii, step t at x = T-1-t - y - z
        VT prev = (VT)0;
        const int lob = rowok ? T - ex - y - z : (1 << 28);
        const int cbb = cb + T - 1;
        for (int t0 = 0; t0 < T; t0 += RB) {
            if (MULTI && w < W - 1) wait_for(&prog[1][w + 1], min(t0 + RB, T));
            VT co[RB][NLP], rin[RB], dg[RB], rz[RB];
            int cc[RB];
            bool aa[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int t = t0 + u;
                aa[u] = (unsigned)(t - lob) < (unsigned)ex;
                cc[u] = min(max(cbb - t, 0), n - 1);
                load_run<FT, VT, NLP>(cf + (size_t)cc[u] * CST + (HALF ? 0 : NLP), co[u]);
                rin[u] = rv[cc[u]];
                dg[u] = (VT)id[cc[u]];
                if (MULTI) rz[u] = rv[min(cc[u] + exy, n - 1)];
            }
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const VT yn = lane_shl(prev);
                VT zn = lane_from(prev, pz_b);
                if (MULTI) zn = zlast ? rz[u] : zn;
                VT v = rin[u];
                v -= co[u][0] * prev;
                v -= co[u][1] * yn;
                v -= co[u][2] * zn;
                prev = aa[u] ? v * dg[u] : (VT)0;
                rv[aa[u] ? cc[u] : n] = prev;
            }
            if (MULTI) __hip_atomic_store(&prog[1][w], t0 + RB, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    if (a.variant == NKS_LEFT_RAS) {
        const int oxn = sd.lx1 - sd.lx0, oyn = sd.ly1 - sd.ly0, ozn = sd.lz1 - sd.lz0;
        const float inv_oxn = 1.0f / (float)oxn, inv_oyn = 1.0f / (float)oyn;
        constexpr int WB = 4;
        const int no = oxn * oyn * ozn;
        for (int k0 = threadIdx.x; k0 < no; k0 += WB * NT) {
            size_t g[WB];
            double v[WB];
#pragma unroll
            for (int u = 0; u < WB; ++u) {
                const int k = min(k0 + u * NT, no - 1);
                const int row = row_of(k, inv_oxn), xx = k - row * oxn;
                const int zz = row_of(row, inv_oyn), yy = row - zz * oyn;
                const int x = sd.lx0 + xx, y = sd.ly0 + yy, z = sd.lz0 + zz;
                g[u] = (size_t)sd.gorg + x + (size_t)sd.gnx * (y + (size_t)sd.gny * z);
                v[u] = (double)rv[x + ex * (y + ey * z)];
            }
            if (a.accumulate) {
#pragma unroll
                for (int u = 0; u < WB; ++u) v[u] += a.z[g[u]];
            }
#pragma unroll
            for (int u = 0; u < WB; ++u)
                if (k0 + u * NT < no) a.z[g[u]] = v[u];
        }
    } else {
        for (int c = threadIdx.x; c < n; c += blockDim.x) a.zext[fo + c] = (double)rv[c];
    }
}

// ---------------------------------------------------------------- kernel: 2D ILU wavefront
// ILU on the factor stencil's pattern (the operator's for ILU(0), with the
// level-of-fill slots for ILU(k); fill slots start at zero) of one 2D box
// per workgroup on the sweeps' schedule: lane y factors
// row y of the box, cell x = t - LB*y at step t, so the row of every lower
// neighbour was finished at an earlier step (by this lane or by a lane
// below).  Rows are staged cell-major in LDS in the row template's slot
// order, then u_ii and 1/u_ii; the row being factored lives in registers.
// IKJ elimination over the lower slots in increasing column order:
// l = a_iq / u_qq (as a product with the stored reciprocal), then
// a_ij -= l u_qj for every upper slot of the neighbour's row whose column is
// a template slot of row i.  Slots absent from the stencil take no
// elimination and are stored as zero, so fill outside the pattern never
// reaches a factor.  Factors are written k-major in lexicographic order,
// straight in their storage precision (off-diagonals FT, 1/u_ii DT),
// rounded from the FP64 elimination.
struct IluRowsArgs {
    const SubDev *sub;
    const Blk *blk;
    const int *slotmap;   // 25 box slots -> factor stencil index or -1
    const int *amap;      // factor stencil index -> operator index (-1: fill, starts at zero)
    const double *A;      // K*N operator
    int N, NE, diag;      // diag: factor stencil index of the diagonal
    void *f;              // K*NE off-diagonal factors, FT (lexicographic per subdomain)
    void *invd;           // NE reciprocal pivots, DT
    int *err;
};

// template slot of offset (dx, dy): NS for the diagonal, -1 outside
template <int BOX>
__host__ __device__ constexpr int row_slot(int dx, int dy) {
    if (dx == 0 && dy == 0) return RowStencil<BOX>::NS;
    for (int q = 0; q < RowStencil<BOX>::NS; ++q)
        if (RowStencil<BOX>::DX[q] == dx && RowStencil<BOX>::DY[q] == dy) return q;
    return -1;
}

// LDS: next * (NS + 2) doubles
template <int BOX, typename FT, typename DT>
__global__ void __launch_bounds__(256) k_ilu_rows(IluRowsArgs a) {
    using S = RowStencil<BOX>;
    constexpr int NS = S::NS, NL = S::NL, LB = S::LB;
    constexpr int RL = NS + 2;   // row length in doubles: off-diagonals, u_ii, 1/u_ii
    static_assert(RL % 2 == 0, "rows are whole 16-byte words");
    extern __shared__ __align__(16) double Wr[];
    __shared__ int kmap[NS + 1];
    const SubDev sd = a.sub[blockIdx.x];
    const Blk bk = a.blk[sd.blk];
    const int n = sd.next, ex = sd.ex, ey = sd.ey;
    if ((int)threadIdx.x <= NS) {
        const int q = threadIdx.x, qq = min(q, NS - 1);
        kmap[q] = q == NS ? a.diag : a.slotmap[(S::DX[qq] + 2) + 5 * (S::DY[qq] + 2)];
    }
    __syncthreads();
    // rows of A_i: neighbours outside the box and absent slots zero
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const int y = c / ex, x = c - y * ex;
        const size_t g = (size_t)bk.off + (sd.ox + x) + (size_t)bk.nx * (sd.oy + y + (size_t)bk.ny * sd.oz);
        double v[NS + 1];
#pragma unroll
        for (int q = 0; q <= NS; ++q) {
            const int dx = q < NS ? S::DX[q] : 0, dy = q < NS ? S::DY[q] : 0;
            const int k = kmap[q] >= 0 ? a.amap[kmap[q]] : -1;
            const bool in = k >= 0 && x + dx >= 0 && x + dx < ex && y + dy >= 0 && y + dy < ey;
            const double av = a.A[(size_t)max(k, 0) * a.N + g];
            v[q] = in ? av : 0.0;
        }
#pragma unroll
        for (int q = 0; q <= NS; ++q) Wr[(size_t)c * RL + q] = v[q];
        Wr[(size_t)c * RL + NS + 1] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int y = threadIdx.x;
        unsigned pm = 0;   // slots present in the stencil (uniform)
#pragma unroll
        for (int q = 0; q < NS; ++q)
            if (kmap[q] >= 0) pm |= 1u << q;
        const int T = (ex - 1) + LB * (ey - 1) + 1;
        int bad = 0;
        for (int t = 0; t < T; ++t) {
            const int x = t - LB * y;
            const bool act = y < ey && x >= 0 && x < ex;
            const int c = act ? y * ex + x : 0;
            double r[NS + 1];
#pragma unroll
            for (int q = 0; q <= NS; ++q) r[q] = Wr[(size_t)c * RL + q];
            // every value of the lower neighbours' rows that the elimination
            // uses is read before the first product (one LDS wait per step);
            // branch-free: every read has a valid (clamped) address
            double ip[NL], ur[NL][NS - NL];
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int ck = min(max(c + S::DX[q] + S::DY[q] * ex, 0), n - 1);
                ip[q] = Wr[(size_t)ck * RL + NS + 1];
#pragma unroll
                for (int p = NL; p < NS; ++p)
                    ur[q][p - NL] = row_slot<BOX>(S::DX[q] + S::DX[p], S::DY[q] + S::DY[p]) >= 0
                                        ? Wr[(size_t)ck * RL + p] : 0.0;
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int xk = x + S::DX[q];
                const bool in = act && ((pm >> q) & 1u) && xk >= 0 && xk < ex && y + S::DY[q] >= 0;
                // an absent neighbour's l is cleared bitwise
                const double l = __longlong_as_double(__double_as_longlong(r[q] * ip[q]) & (in ? ~0ll : 0ll));
                r[q] = l;
#pragma unroll
                for (int p = NL; p < NS; ++p) {
                    const int tg = row_slot<BOX>(S::DX[q] + S::DX[p], S::DY[q] + S::DY[p]);
                    if (tg < 0) continue;
                    r[tg] -= l * ur[q][p - NL];
                }
            }
            const double u = r[NS];
            if (act) {
                if (!(u != 0.0) || !isfinite(u)) bad = 1;
#pragma unroll
                for (int q = 0; q < NS; ++q) Wr[(size_t)c * RL + q] = ((pm >> q) & 1u) ? r[q] : 0.0;
                Wr[(size_t)c * RL + NS] = u;
                Wr[(size_t)c * RL + NS + 1] = 1.0 / u;
            }
            // the next step reads rows that lanes of this wavefront wrote
            // above: LDS operations of one wavefront complete in order, the
            // fences keep the compiler from moving reads above those writes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (bad) atomicOr(a.err, 1);
    }
    __syncthreads();
    // factors out, k-major, cells contiguous; the diagonal as 1/u_ii
    const size_t fo = sd.fac_off;
    FT *F = reinterpret_cast<FT *>(a.f);
    DT *ID = reinterpret_cast<DT *>(a.invd);
    for (int i = threadIdx.x; i < NS * n; i += blockDim.x) {
        const int q = i / n, c = i - q * n;
        const int k = kmap[q];
        if (k < 0) continue;
        const double v = Wr[(size_t)c * RL + q];
        if constexpr (sizeof(FT) == 2) F[(size_t)k * a.NE + fo + c] = to_bf16((float)v);
        else F[(size_t)k * a.NE + fo + c] = (FT)v;
    }
    for (int c = threadIdx.x; c < n; c += blockDim.x) ID[fo + c] = (DT)Wr[(size_t)c * RL + NS + 1];
}

// AS / right-RAS: z_g = sum over the boxes whose extension holds g (box order)
__device__ __forceinline__ int box_of(int x, int n, int P) {
    const int base = n / P, rem = n % P;
    const int big = rem * (base + 1);
    return x < big ? x / (base + 1) : rem + (x - big) / base;
}

__global__ void k_ras_gather(const Blk *blk, int B, int N, const BlkPart *part, const SubDev *sub,
                             const double *zext, double *z, const int *mask, int accumulate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = find_blk(blk, B, i);
    if (mask && !mask[b]) return;
    const Blk k = blk[b];
    const BlkPart P = part[b];
    const int l = i - k.off;
    const int x = l % k.nx, y = (l / k.nx) % k.ny, zz = l / (k.nx * k.ny);
    const int qx = box_of(x, k.nx, P.px), qy = box_of(y, k.ny, P.py), qz = box_of(zz, k.nz, P.pz);
    double s = 0.0;
    for (int cz = qz - 1; cz <= qz + 1; ++cz) {
        if (cz < 0 || cz >= P.pz) continue;
        for (int cy = qy - 1; cy <= qy + 1; ++cy) {
            if (cy < 0 || cy >= P.py) continue;
            for (int cx = qx - 1; cx <= qx + 1; ++cx) {
                if (cx < 0 || cx >= P.px) continue;
                const SubDev sd = sub[P.first + cx + P.px * (cy + P.py * cz)];
                const int lx = x - sd.ox, ly = y - sd.oy, lz = zz - sd.oz;
                if (lx < 0 || lx >= sd.ex || ly < 0 || ly >= sd.ey || lz < 0 || lz >= sd.ez) continue;
                s += zext[sd.fac_off + lx + sd.ex * (ly + sd.ey * lz)];
            }
        }
    }
    z[i] = accumulate ? z[i] + s : s;
}

// ---------------------------------------------------------------- kernels: grid transfer
struct XferArgs {
    const Blk *fblk, *cblk;
    int B, Nf, Nc;
    const int *rcnt[3], *rj[3], *ccnt[3], *ci[3], *roff[3], *coff[3];
    const double *rw[3], *cw[3];
    int cs[3];            // column stride of ci / cw per direction
    const int *mask;
};

// r_c = P^T r_f (gather over the fine support of each coarse cell).  The
// x list of the coarse column sits in registers (up to XM entries) so that a
// fine row's loads go out together; longer lists take the plain loops.
// A workgroup per tile of the coarse level (a run of at most TILE cells of
// one reservoir), so the reservoir comes with the tile.
// XM is 8 or 16, the smallest that holds the level's longest x column.
template <int XM>
__device__ __forceinline__ void restrict_cell(const XferArgs &a, int b, const Blk &cb, const Blk &fb, int I,
                                              const double *rf, double *rc) {
    const int l = I - cb.off;
    const int X = l % cb.nx, Y = (l / cb.nx) % cb.ny, Z = l / (cb.nx * cb.ny);
    const int cx = a.coff[0][b] + X, cy = a.coff[1][b] + Y, cz = a.coff[2][b] + Z;
    const int nqx = a.ccnt[0][cx];
    double s = 0.0;
    if (nqx <= XM) {
        int fxs[XM];
        double wxs[XM];
#pragma unroll
        for (int q = 0; q < XM; ++q) {
            const int qq = max(0, min(q, nqx - 1));
            fxs[q] = a.ci[0][cx * a.cs[0] + qq];
            wxs[q] = q < nqx ? a.cw[0][cx * a.cs[0] + qq] : 0.0;
        }
        // a 2D reservoir's z column is the single entry (0, 1): not loaded
        const bool flat = fb.nz == 1;
        const int nqz = flat ? 1 : a.ccnt[2][cz];
        for (int qz = 0; qz < nqz; ++qz) {
            const int fz = flat ? 0 : a.ci[2][cz * a.cs[2] + qz];
            const double wz = flat ? 1.0 : a.cw[2][cz * a.cs[2] + qz];
            for (int qy = 0; qy < a.ccnt[1][cy]; ++qy) {
                const int fy = a.ci[1][cy * a.cs[1] + qy];
                const double wyz = a.cw[1][cy * a.cs[1] + qy] * wz;
                const double *row = rf + fb.off + (size_t)fb.nx * (fy + (size_t)fb.ny * fz);
                double v[XM];
#pragma unroll
                for (int q = 0; q < XM; ++q) v[q] = q < nqx ? row[fxs[q]] : 0.0;
#pragma unroll
                for (int q = 0; q < XM; ++q)
                    if (q < nqx) s += (wxs[q] * wyz) * v[q];
            }
        }
        rc[I] = s;
        return;
    }
    for (int qz = 0; qz < a.ccnt[2][cz]; ++qz) {
        const int fz = a.ci[2][cz * a.cs[2] + qz];
        const double wz = a.cw[2][cz * a.cs[2] + qz];
        for (int qy = 0; qy < a.ccnt[1][cy]; ++qy) {
            const int fy = a.ci[1][cy * a.cs[1] + qy];
            const double wy = a.cw[1][cy * a.cs[1] + qy];
            for (int qx = 0; qx < nqx; ++qx) {
                const int fx = a.ci[0][cx * a.cs[0] + qx];
                const double wx = a.cw[0][cx * a.cs[0] + qx];
                s += (wx * wy * wz) * rf[fb.off + fx + fb.nx * (fy + fb.ny * fz)];
            }
        }
    }
    rc[I] = s;
}

template <int XM>
__global__ void k_restrict(XferArgs a, const Chunk *chunks, const double *rf, double *rc) {
    const Chunk ch = chunks[blockIdx.x];
    const int b = ch.blk;
    if (a.mask && !a.mask[b]) return;
    const Blk cb = a.cblk[b], fb = a.fblk[b];
    for (int I = ch.start + (int)threadIdx.x; I < ch.end; I += blockDim.x)
        restrict_cell<XM>(a, b, cb, fb, I, rf, rc);
}

// z_f += P e_c: rows of P hold at most four entries per direction, all
// loaded before the sum; a workgroup per tile of the fine level
__device__ __forceinline__ void prolong_cell(const XferArgs &a, int b, const Blk &cb, const Blk &fb, int i,
                                             const double *ec, double *zf) {
    const int l = i - fb.off;
    const int x = l % fb.nx, y = (l / fb.nx) % fb.ny, z = l / (fb.nx * fb.ny);
    const int rx = a.roff[0][b] + x, ry = a.roff[1][b] + y, rz = a.roff[2][b] + z;
    int n[3], J[3][4];
    double w[3][4];
    const int r[3] = {rx, ry, rz};
    // a 2D reservoir's z row is the single entry (0, 1): not loaded
    const int nd = fb.nz == 1 ? 2 : 3;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d < nd) {
            n[d] = a.rcnt[d][r[d]];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                J[d][q] = a.rj[d][r[d] * 4 + q];
                w[d][q] = a.rw[d][r[d] * 4 + q];
            }
        } else {
            n[d] = 1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                J[d][q] = 0;
                w[d][q] = q == 0 ? 1.0 : 0.0;
            }
        }
    }
    const double zi = zf[i];
    double s = 0.0;
#pragma unroll
    for (int qz = 0; qz < 4; ++qz) {
        if (qz >= n[2]) break;
#pragma unroll
        for (int qy = 0; qy < 4; ++qy) {
            if (qy >= n[1]) break;
            const double wyz = w[2][qz] * w[1][qy];
            const double *row = ec + cb.off + (size_t)cb.nx * (J[1][qy] + (size_t)cb.ny * J[2][qz]);
            double v[4];
#pragma unroll
            for (int qx = 0; qx < 4; ++qx) v[qx] = row[qx < n[0] ? J[0][qx] : J[0][0]];
#pragma unroll
            for (int qx = 0; qx < 4; ++qx)
                if (qx < n[0]) s += (w[0][qx] * wyz) * v[qx];
        }
    }
    zf[i] = zi + s;
}

__global__ void k_prolong_add(XferArgs a, const Chunk *chunks, const double *ec, double *zf) {
    const Chunk ch = chunks[blockIdx.x];
    const int b = ch.blk;
    if (a.mask && !a.mask[b]) return;
    const Blk cb = a.cblk[b], fb = a.fblk[b];
    for (int i = ch.start + (int)threadIdx.x; i < ch.end; i += blockDim.x) prolong_cell(a, b, cb, fb, i, ec, zf);
}

// Galerkin A_c = P^T A P, one wavefront per coarse cell I: the lanes share
// the fine cells f of I's interpolation support (the column of P), each lane
// adding P(f,I) A(f,g) P(g,J) into its own LDS row of Kc slots (slot of the
// offset J - I); then lane k sums slot k over the wavefront's 64 rows in a
// fixed order, so the product is deterministic.  The tables a lane walks per
// term (P rows of g, the offset-to-slot map) are read through the per-block
// LDS copy of the slot map and a handful of global loads per fine cell.
template <int W>
__global__ void __launch_bounds__(64 * W) k_rap(XferArgs a, const double *Af, int Kf, const int8_t *offf,
                                                double *Ac, int Kc, const int *slot, int Rc) {
    extern __shared__ double rap_s[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int S = 2 * Rc + 1, S3 = S * S * S;
    int *slot_s = reinterpret_cast<int *>(rap_s + (size_t)64 * W * Kc);
    for (int t = threadIdx.x; t < S3; t += 64 * W) slot_s[t] = slot[t];
    double *acc = rap_s + (size_t)threadIdx.x * Kc;
    for (int k = 0; k < Kc; ++k) acc[k] = 0.0;
    __syncthreads();
    const int I = blockIdx.x * W + w;
    int b = 0, X = 0, Y = 0, Z = 0;
    if (I < a.Nc) {
        b = find_blk(a.cblk, a.B, I);
        const Blk cb = a.cblk[b], fb = a.fblk[b];
        const int l = I - cb.off;
        X = l % cb.nx;
        Y = (l / cb.nx) % cb.ny;
        Z = l / (cb.nx * cb.ny);
        const int cx = a.coff[0][b] + X, cy = a.coff[1][b] + Y, cz = a.coff[2][b] + Z;
        const int nqx = a.ccnt[0][cx], nqy = a.ccnt[1][cy], nqz = a.ccnt[2][cz];
        const int tot = nqx * nqy * nqz;
        for (int q = lane; q < tot; q += 64) {
            const int qx = q % nqx, qy = (q / nqx) % nqy, qz = q / (nqx * nqy);
            const int fx = a.ci[0][cx * a.cs[0] + qx], fy = a.ci[1][cy * a.cs[1] + qy],
                      fz = a.ci[2][cz * a.cs[2] + qz];
            const double wf = a.cw[0][cx * a.cs[0] + qx] * a.cw[1][cy * a.cs[1] + qy] * a.cw[2][cz * a.cs[2] + qz];
            const int f = fb.off + fx + fb.nx * (fy + fb.ny * fz);
            for (int k = 0; k < Kf; ++k) {
                const int gx = fx + offf[3 * k], gy = fy + offf[3 * k + 1], gz = fz + offf[3 * k + 2];
                if (gx < 0 || gx >= fb.nx || gy < 0 || gy >= fb.ny || gz < 0 || gz >= fb.nz) continue;
                const double av = Af[(size_t)k * a.Nf + f];
                if (av == 0.0) continue;
                const double wa = wf * av;
                const int rx = a.roff[0][b] + gx, ry = a.roff[1][b] + gy, rz = a.roff[2][b] + gz;
                const int npx = a.rcnt[0][rx], npy = a.rcnt[1][ry], npz = a.rcnt[2][rz];
                for (int pz = 0; pz < npz; ++pz) {
                    const int Jz = a.rj[2][rz * 4 + pz];
                    const double vz = wa * a.rw[2][rz * 4 + pz];
                    for (int py = 0; py < npy; ++py) {
                        const int Jy = a.rj[1][ry * 4 + py];
                        const double vyz = vz * a.rw[1][ry * 4 + py];
                        const int row = S * ((Jy - Y + Rc) + S * (Jz - Z + Rc)) + Rc - X;
                        for (int px = 0; px < npx; ++px) {
                            const int sl = slot_s[row + a.rj[0][rx * 4 + px]];
                            acc[sl] += vyz * a.rw[0][rx * 4 + px];
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    if (I < a.Nc) {
        const double *rows = rap_s + (size_t)w * 64 * Kc;
        for (int k = lane; k < Kc; k += 64) {
            double sum = 0.0;
            for (int r = 0; r < 64; ++r) sum += rows[(size_t)r * Kc + k];
            Ac[(size_t)k * a.Nc + I] = sum;
        }
    }
}

// Galerkin A_c = P^T A P on 2D levels, one wavefront per coarse column J:
// first AP(f, J) = sum_k A(f, f + o_k) P(f + o_k, J) over the window of
// fine cells f that reach J's interpolation support, then every entry of
// the column, A_c(I, J) = sum_f P(f, I) AP(f, J) for I = J - o over the
// coarse stencil offsets o, with the tensor weights
// P(f, I) = p_x(f_x, I_x) p_y(f_y, I_y) summed one direction at a time:
// U(o_x, f_y) = sum_{f_x} p_x(f_x, J_x - o_x) AP(f_x, f_y), then
// A_c(J - o, J) = sum_{f_y} p_y(f_y, J_y - o_y) U(o_x, f_y).  Every sum runs
// in a fixed order, so the product is deterministic.  Each entry of A_c is
// written by the wavefront of its column; entries whose column lies outside
// the block stay as the caller zeroed them.
struct Rap2Lds {
    int wg[2], wx, wy, per;   // table widths (window + reach) and doubles per wavefront
};
__host__ __device__ inline Rap2Lds rap2_lds(int wx, int wy, int Rf, int Rc) {
    Rap2Lds L;
    L.wx = wx;
    L.wy = wy;
    L.wg[0] = wx + 2 * Rf;
    L.wg[1] = wy + 2 * Rf;
    const int nc = 2 * Rc + 1;
    L.per = nc * (L.wg[0] + L.wg[1]) + wx * wy + nc * wy;
    return L;
}

struct Rap2Tabs {
    const int4 *cell;
    const int2 *win[2];
    const double *tab[2];
};

// KM: the fine stencil's compile-time bound (its loads for a cell go out
// together; a 5-point operator keeps its registers, and its occupancy, low)
template <int W, int KM>
__global__ void __launch_bounds__(64 * W) k_rap2d(XferArgs a, Rap2Tabs tb, const double *Af, int Kf,
                                                  const int8_t *offf, int Rf, double *Ac, int Kc, const int8_t *offc,
                                                  int Rc, int wxm, int wym) {
    extern __shared__ double rap2_s[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const Rap2Lds L = rap2_lds(wxm, wym, Rf, Rc);
    const int nc = 2 * Rc + 1;
    double *Tx = rap2_s + (size_t)w * L.per;        // [o][f_x - (wx0 - Rf)]: p_x(f_x, J_x - (o - Rc))
    double *Ty = Tx + nc * L.wg[0];
    double *AP = Ty + nc * L.wg[1];                 // [f_y - wy0][f_x - wx0]
    double *U = AP + L.wx * L.wy;                   // [o_x + Rc][f_y - wy0]
    const int J = blockIdx.x * W + w;
    const bool on = J < a.Nc;
    int4 ci = make_int4(0, 0, 0, 0);
    int2 wxn = make_int2(0, 0), wyn = make_int2(0, 0);
    Blk cb{}, fb{};
    if (on) {
        ci = tb.cell[J];
        cb = a.cblk[ci.x];
        fb = a.fblk[ci.x];
        wxn = tb.win[0][ci.y];
        wyn = tb.win[1][ci.z];
        // the column's weight tables, as laid out in memory
        const double *gx = tb.tab[0] + (size_t)ci.y * nc * L.wg[0];
        const double *gy = tb.tab[1] + (size_t)ci.z * nc * L.wg[1];
        for (int t = lane; t < nc * L.wg[0]; t += 64) Tx[t] = gx[t];
        for (int t = lane; t < nc * L.wg[1]; t += 64) Ty[t] = gy[t];
    }
    const int Jx = ci.w & 0xffff, Jy = ci.w >> 16;
    const int wx0 = wxn.x, WX = wxn.y, wy0 = wyn.x, WY = wyn.y;
    __syncthreads();
    if (on) {
        // AP over the window.  A's coefficients towards neighbours outside
        // the block are zero and the tables are zero off the supports (which
        // lie inside the block), so no term needs a bounds test: the Kf
        // loads of a cell go out together.
        const double *TJx = Tx + Rc * L.wg[0], *TJy = Ty + Rc * L.wg[1];
        for (int t = lane; t < WX * WY; t += 64) {
            const int ux = t % WX, uy = t / WX;
            const int fx = wx0 + ux, fy = wy0 + uy;
            const size_t f = (size_t)fb.off + fx + (size_t)fb.nx * fy;
            double av[KM];
#pragma unroll
            for (int k = 0; k < KM; ++k) av[k] = k < Kf ? Af[(size_t)k * a.Nf + f] : 0.0;
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (k < Kf) {
                    const int gx = ux + Rf + offf[3 * k], gy = uy + Rf + offf[3 * k + 1];
                    s += av[k] * (TJx[gx] * TJy[gy]);
                }
            }
            AP[uy * L.wx + ux] = s;
        }
    }
    __syncthreads();
    if (on) {
        for (int t = lane; t < nc * WY; t += 64) {
            const int o = t / WY, uy = t % WY;
            const double *tx = Tx + o * L.wg[0] + Rf;
            double s = 0.0;
            for (int ux = 0; ux < WX; ++ux) s += tx[ux] * AP[uy * L.wx + ux];
            U[o * L.wy + uy] = s;
        }
    }
    __syncthreads();
    if (on) {
        for (int k = lane; k < Kc; k += 64) {
            const int ox = offc[3 * k], oy = offc[3 * k + 1];
            const int Ix = Jx - ox, Iy = Jy - oy;
            if (Ix < 0 || Ix >= cb.nx || Iy < 0 || Iy >= cb.ny) continue;
            const double *ty = Ty + (oy + Rc) * L.wg[1] + Rf;
            double s = 0.0;
            for (int uy = 0; uy < WY; ++uy) s += ty[uy] * U[(ox + Rc) * L.wy + uy];
            Ac[(size_t)k * a.Nc + cb.off + Ix + (size_t)cb.nx * Iy] = s;
        }
    }
}

__global__ void k_fill(int N, double v, double *x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) x[i] = v;
}

// ---------------------------------------------------------------- host: hierarchy
static XferArgs xfer_args(Level &F, Level &C, const int *mask) {
    XferArgs a;
    a.fblk = F.spp->blk.p;
    a.cblk = C.spp->blk.p;
    a.B = F.spp->B;
    a.Nf = F.spp->N;
    a.Nc = C.spp->N;
    for (int d = 0; d < 3; ++d) {
        a.rcnt[d] = F.ip[d].d_rcnt.p;
        a.rj[d] = F.ip[d].d_rj.p;
        a.rw[d] = F.ip[d].d_rw.p;
        a.ccnt[d] = F.ip[d].d_ccnt.p;
        a.ci[d] = F.ip[d].d_ci.p;
        a.cw[d] = F.ip[d].d_cw.p;
        a.roff[d] = F.ip[d].d_roff.p;
        a.coff[d] = F.ip[d].d_coff.p;
        a.cs[d] = F.ip[d].cs;
    }
    a.mask = mask;
    return a;
}

// LDS of the row sweep over the largest box of a 2D level in the given precision
template <typename FT, typename VT, typename DT>
static size_t rows_sweep_lds_t(const Level &V) {
    const int cs = V.box == 0 ? row_stride<0, FT>() : (V.box == 1 ? row_stride<1, FT>() : row_stride<2, FT>());
    return rows_lds(sizeof(VT), sizeof(FT), sizeof(DT), cs, rows_pad(V.box), (size_t)V.max_next).total;
}
static size_t rows_sweep_lds(const Level &V, int precision) {
    if (precision == NKS_FP64) return rows_sweep_lds_t<double, double, double>(V);
    if (precision == NKS_FP32) return rows_sweep_lds_t<float, float, float>(V);
    return rows_sweep_lds_t<uint16_t, float, float>(V);
}

// Groups for the packed sweep of a 2D level: consecutive boxes of one
// block, their rows filling at most 64 lanes and their runs at most half
// the LDS (two groups per CU).  Levels whose groups would average fewer
// than two boxes keep one box per workgroup.
template <int BOX, typename FT>
static size_t packed_group_lds(int precision, size_t n) {
    const size_t vt = precision == NKS_FP64 ? 8 : 4;
    return packed_lds(vt, sizeof(FT), vt, row_stride<BOX, FT>(), BOX, n).total;
}
static size_t packed_group_lds(const Level &V, int precision, size_t n) {
    if (precision == NKS_FP64)
        return V.box == 0 ? packed_group_lds<0, double>(precision, n)
                          : (V.box == 1 ? packed_group_lds<1, double>(precision, n) : packed_group_lds<2, double>(precision, n));
    if (precision == NKS_FP32)
        return V.box == 0 ? packed_group_lds<0, float>(precision, n)
                          : (V.box == 1 ? packed_group_lds<1, float>(precision, n) : packed_group_lds<2, float>(precision, n));
    return V.box == 0 ? packed_group_lds<0, uint16_t>(precision, n)
                      : (V.box == 1 ? packed_group_lds<1, uint16_t>(precision, n)
                                    : packed_group_lds<2, uint16_t>(precision, n));
}

static void build_packed(Level &V, int precision, int lds_bytes, Alloc *al, hipStream_t s) {
    V.pk_groups = 0;
    V.pk_max_n = 0;
    if (!V.rows2d || V.nsub == 0) return;
    const int LB = V.box == 0 ? RowStencil<0>::LB : (V.box == 1 ? RowStencil<1>::LB : RowStencil<2>::LB);
    const size_t budget = (size_t)lds_bytes / 2;
    std::vector<int2> lane;
    std::vector<int> steps, first;
    size_t max_n = 0;
    int used = 64, blk = -1;
    size_t n = 0;
    for (int q = 0; q < V.nsub; ++q) {
        const SubDev &sd = V.hsub[q];
        if (sd.ez != 1 || sd.ey > 64) return;
        if (q > 0 && sd.fac_off != V.hsub[q - 1].fac_off + V.hsub[q - 1].next) return;
        if (used + sd.ey > 64 || sd.blk != blk || packed_group_lds(V, precision, n + sd.next) > budget) {
            lane.resize(lane.size() + 64, int2{q, -1});
            steps.push_back(0);
            first.push_back(q);
            used = 0;
            n = 0;
            blk = sd.blk;
        }
        const size_t g = steps.size() - 1;
        for (int y = 0; y < sd.ey; ++y) lane[g * 64 + used + y] = int2{q, y};
        used += sd.ey;
        n += sd.next;
        max_n = std::max(max_n, n);
        steps[g] = std::max(steps[g], (sd.ex - 1) + LB * (sd.ey - 1) + 1);
    }
    const int G = (int)steps.size();
    if (2 * G > V.nsub || packed_group_lds(V, precision, max_n) > (size_t)lds_bytes) return;
    first.push_back(V.nsub);
    std::vector<int> e2g(V.next_total, 0);
    for (const SubDev &sd : V.hsub)
        for (int y = 0; y < sd.ey; ++y)
            for (int x = 0; x < sd.ex; ++x) {
                const bool own = x >= sd.lx0 && x < sd.lx1 && y >= sd.ly0 && y < sd.ly1;
                const long gc = (long)sd.gorg + x + (long)sd.gnx * y;
                e2g[sd.fac_off + x + sd.ex * y] = (int)gc | (own ? (int)0x80000000u : 0);
            }
    V.pk_lane.upload(al, lane, s);
    V.pk_steps.upload(al, steps, s);
    V.pk_box.upload(al, first, s);
    V.pk_e2g.upload(al, e2g, s);
    V.pk_groups = G;
    V.pk_max_n = max_n;
}

// Tables of the column-wise 2D Galerkin product (see k_rap2d)
static void build_rap_tables(Level &F, Level &C, const std::vector<int> &nfx, const std::vector<int> &nfy, int Rf,
                             int Rc, Alloc *al, hipStream_t s) {
    const int nc = 2 * Rc + 1;
    const std::vector<int> *nfs[2] = {&nfx, &nfy};
    for (int d = 0; d < 2; ++d) {
        const Interp1 &ip = F.ip[d];
        const int wg = (d == 0 ? F.rap_wx : F.rap_wy) + 2 * Rf;
        const int ncols = (int)ip.ccnt.size();
        std::vector<int2> win(ncols, int2{0, 0});
        std::vector<double> tab((size_t)ncols * nc * wg, 0.0);
        for (size_t b = 0; b < nfs[d]->size(); ++b) {
            const int nf = (*nfs[d])[b], c0 = ip.coff[b];
            const int ncb = (b + 1 < nfs[d]->size() ? ip.coff[b + 1] : ncols) - c0;
            for (int Ic = 0; Ic < ncb; ++Ic) {
                const int c = c0 + Ic;
                if (ip.ccnt[c] < 1) continue;
                const int lo = ip.ci[(size_t)c * ip.cs], hi = ip.ci[(size_t)c * ip.cs + ip.ccnt[c] - 1];
                const int w0 = std::max(0, lo - Rf);
                win[c] = int2{w0, std::min(nf, hi + Rf + 1) - w0};
                for (int o = 0; o < nc; ++o) {
                    const int Io = Ic - (o - Rc);
                    if (Io < 0 || Io >= ncb) continue;
                    const int co = c0 + Io;
                    for (int q = 0; q < ip.ccnt[co]; ++q) {
                        const int k = ip.ci[(size_t)co * ip.cs + q] - (w0 - Rf);
                        if (k >= 0 && k < wg) tab[((size_t)c * nc + o) * wg + k] = ip.cw[(size_t)co * ip.cs + q];
                    }
                }
            }
        }
        F.rap_win[d].upload(al, win, s);
        F.rap_tab[d].upload(al, tab, s);
    }
    std::vector<int4> cell(C.spp->N);
    for (int b = 0; b < C.spp->B; ++b) {
        const Blk &k = C.spp->hblk[b];
        for (int y = 0; y < k.ny; ++y)
            for (int x = 0; x < k.nx; ++x)
                cell[k.off + x + k.nx * y] = int4{b, F.ip[0].coff[b] + x, F.ip[1].coff[b] + y, x | (y << 16)};
    }
    F.rap_cell.upload(al, cell, s);
}

void Ras::build(Matrix *Jm, const nks_ras_desc &dd) {
    J = Jm;
    g = Jm->g;
    d = dd;
    L = std::max(1, std::min(d.levels, 6));
    Alloc *al = &g->al;
    hipStream_t s = g->s;
    coarse.invalidate_graphs();
    lev.clear();
    tiles_.clear();
    lev.emplace_back(new Level());
    lev[0]->spp = &g->sp;
    lev[0]->A = &Jm->op;
    const int rt = d.ratio > 0 ? d.ratio : 2;
    for (int l = 0; l + 1 < L; ++l) {
        Level &F = *lev[l];
        lev.emplace_back(new Level());
        Level &C = *lev[l + 1];
        std::vector<Blk> cb;
        std::vector<int> nfx, nfy, nfz;
        for (const Blk &k : F.spp->hblk) {
            cb.push_back({k.nx > 1 ? (k.nx + rt - 1) / rt : 1, k.ny > 1 ? (k.ny + rt - 1) / rt : 1,
                          k.nz > 1 ? (k.nz + rt - 1) / rt : 1, 0});
            nfx.push_back(k.nx);
            nfy.push_back(k.ny);
            nfz.push_back(k.nz);
        }
        build_interp(F.ip[0], nfx, d.interp_order, rt, al, s);
        build_interp(F.ip[1], nfy, d.interp_order, rt, al, s);
        build_interp(F.ip[2], nfz, d.interp_order, rt, al, s);
        if (d.coarse_op == NKS_COARSE_REDISCRETIZED) {
            // the coarse matrix is the Jacobian of the upscaled problem: the
            // fine stencil on the coarse grid's own space
            C.cg.reset(new Grid());
            coarsen_grid(l == 0 ? *g : *F.cg, rt, *C.cg);
            C.spp = &C.cg->sp;
            C.cstate.alloc(al, C.spp->N);
            C.own.sp = C.spp;
            std::vector<std::tuple<int, int, int>> offs;
            for (int k = 0; k < F.A->st.K; ++k)
                offs.push_back({F.A->st.off[3 * k], F.A->st.off[3 * k + 1], F.A->st.off[3 * k + 2]});
            set_stencil(C.own.st, offs, al, s);
            C.own.coef.alloc(al, (size_t)C.own.st.K * C.spp->N);
            C.A = &C.own;
            continue;
        }
        C.sp.build(al, cb, s);
        C.spp = &C.sp;
        // coarse stencil: union over fine offsets of the tensor 1D coupling sets
        const Stencil &fs = F.A->st;
        std::set<std::tuple<int, int, int>> offs;
        std::map<int, std::set<int>> cx, cy, cz;
        for (int k = 0; k < fs.K; ++k) {
            const int ox = fs.off[3 * k], oy = fs.off[3 * k + 1], oz = fs.off[3 * k + 2];
            if (!cx.count(ox)) cx[ox] = coupling_1d(F.ip[0], nfx, ox);
            if (!cy.count(oy)) cy[oy] = coupling_1d(F.ip[1], nfy, oy);
            if (!cz.count(oz)) cz[oz] = coupling_1d(F.ip[2], nfz, oz);
            for (int a : cx[ox])
                for (int b : cy[oy])
                    for (int c : cz[oz]) offs.insert({a, b, c});
        }
        offs.insert({0, 0, 0});
        C.own.sp = &C.sp;
        set_stencil(C.own.st, std::vector<std::tuple<int, int, int>>(offs.begin(), offs.end()), al, s);
        C.own.coef.alloc(al, (size_t)C.own.st.K * C.sp.N);
        C.A = &C.own;
        // slot table for the Galerkin kernel
        const int Rc = C.own.st.R, S = 2 * Rc + 1;
        std::vector<int> slot(S * S * S, 0);
        for (int k = 0; k < C.own.st.K; ++k)
            slot[(C.own.st.off[3 * k] + Rc) + S * ((C.own.st.off[3 * k + 1] + Rc) + S * (C.own.st.off[3 * k + 2] + Rc))] = k;
        F.rap_slot.upload(al, slot, s);
        F.rap_R = Rc;
        // 2D: windows of the column-wise product (J's support widened by the
        // fine stencil's reach)
        bool flat = fs.R >= 0;
        for (const Blk &k : F.spp->hblk) flat = flat && k.nz == 1;
        for (int k = 0; k < fs.K; ++k) flat = flat && fs.off[3 * k + 2] == 0;
        F.rap_wx = F.rap_wy = 0;
        if (flat) {
            for (int d = 0; d < 2; ++d) {
                const Interp1 &ip = F.ip[d];
                int wmax = 0;
                for (size_t c = 0; c < ip.ccnt.size(); ++c) {
                    if (ip.ccnt[c] < 1) continue;
                    const int lo = ip.ci[c * ip.cs], hi = ip.ci[c * ip.cs + ip.ccnt[c] - 1];
                    wmax = std::max(wmax, hi - lo + 1 + 2 * fs.R);
                }
                (d == 0 ? F.rap_wx : F.rap_wy) = wmax;
            }
            build_rap_tables(F, C, nfx, nfy, fs.R, Rc, al, s);
        }
    }
    // the same box grid on every level: box counts per reservoir from the finest level
    std::vector<std::array<int, 3>> boxes;
    for (const Blk &k : lev[0]->spp->hblk) {
        const int t[3] = {d.tx, d.ty, d.tz}, n[3] = {k.nx, k.ny, k.nz}, p[3] = {d.px, d.py, d.pz};
        std::array<int, 3> bx;
        for (int a = 0; a < 3; ++a) bx[a] = t[a] > 0 ? (n[a] + t[a] - 1) / t[a] : p[a];
        boxes.push_back(bx);
    }
    for (int l = 0; l < L; ++l) {
        Level &V = *lev[l];
        TileDims geo;
        std::vector<int> amap;
        factor_stencil(V.A->st, d.fill, V.fst, amap, al, s);
        V.amap.upload(al, amap, s);
        build_partition(V, boxes, d.overlap[std::min(l, 7)], al, s, geo);
        const size_t NE = V.next_total, K = V.fst.K;
        V.w64.alloc(al, K * NE);
        if (d.precision == NKS_FP64) {
            V.invd64.alloc(al, NE);
            V.f64.alloc(al, K * NE);
        } else {
            V.invd32.alloc(al, NE);
            if (d.precision == NKS_FP32) V.f32.alloc(al, K * NE);
            else V.f16.alloc(al, K * NE);
        }
        if (d.variant != NKS_LEFT_RAS) V.zext.alloc(al, NE);
        V.r.alloc(al, V.spp->N);
        V.t.alloc(al, V.spp->N);
        V.bc.alloc(al, V.spp->N);
        V.xc.alloc(al, V.spp->N);
        // geometry for kernels kept in hsub / lin_pad; remember tile dims
        tiles_.push_back(geo);
    }
    // the coarse GMRES keeps M v_j per iteration (see coarse_solve)
    if (L > 1) coarse.ensure(al, *lev[L - 1]->spp, std::max(1, std::min(d.coarse_restart, 30)), true, s);
    int dev = 0, maxlds = 65536;
    HIPC(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        maxlds = 65536;
    lds_bytes = std::min(maxlds, 160 * 1024);
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
        n_cu = 1;
    // a 2D level whose boxes do not fit the row sweep's LDS (ILU(k) fill
    // widens a cell's run) takes the hyperplane kernels
    for (auto &V : lev)
        if (V->rows2d && rows_sweep_lds(*V, d.precision) > (size_t)lds_bytes) V->rows2d = false;
    for (auto &V : lev) build_packed(*V, d.precision, lds_bytes, al, s);
    setup_persistent();
}

static bool use_rows3d(const Ras &M, const Level &V);

void Ras::factor(bool ilu) {
    hipStream_t s = g->s;
    const bool redisc = d.coarse_op == NKS_COARSE_REDISCRETIZED && L > 1;
    if (redisc && !J->has_state)
        fail(NKS_EINVAL, "rediscretised coarse levels need the state of the Jacobian (nks_jacobian)");
    for (int l = 0; l < L; ++l) {
        Level &V = *lev[l];
        if (l > 0 && redisc) {
            // coarsened state, then the upscaled problem's Jacobian at it
            const Grid &fg = l == 1 ? *g : *lev[l - 1]->cg;
            const double *pf = l == 1 ? J->state.p : lev[l - 1]->cstate.p;
            launch_coarsen_mean(fg, *V.cg, pf, V.cstate.p);
            launch_props(*V.cg, V.cstate.p);
            launch_flux(*V.cg, V.cstate.p, J->dt, J->order, nullptr, V.own.coef.p);
        } else if (l > 0 && lev[l - 1]->rap_wx > 0 && lev[l - 1]->A->st.K <= 25 &&
                   (size_t)rap2_lds(lev[l - 1]->rap_wx, lev[l - 1]->rap_wy, lev[l - 1]->A->st.R, lev[l - 1]->rap_R).per *
                           sizeof(double) <= (size_t)lds_bytes) {
            Level &F = *lev[l - 1];
            XferArgs a = xfer_args(F, V, nullptr);
            const int Kc = V.own.st.K, Nc = V.spp->N;
            const size_t per = (size_t)rap2_lds(F.rap_wx, F.rap_wy, F.A->st.R, F.rap_R).per * sizeof(double);
            const int W = 4 * per <= (size_t)lds_bytes ? 4 : (2 * per <= (size_t)lds_bytes ? 2 : 1);
            k_fill<<<nblk((int)std::min<size_t>((size_t)Kc * Nc, INT32_MAX), 256), 256, 0, s>>>(Kc * Nc, 0.0,
                                                                                               V.own.coef.p);
            KCHECK();
            Rap2Tabs tb{F.rap_cell.p, {F.rap_win[0].p, F.rap_win[1].p}, {F.rap_tab[0].p, F.rap_tab[1].p}};
            using RapFn = void (*)(XferArgs, Rap2Tabs, const double *, int, const int8_t *, int, double *, int,
                                   const int8_t *, int, int, int);
            auto pick = [&](auto km) -> RapFn {
                constexpr int KM = decltype(km)::value;
                return W == 4 ? k_rap2d<4, KM> : (W == 2 ? k_rap2d<2, KM> : k_rap2d<1, KM>);
            };
            const int Kf = F.A->st.K;
            RapFn fr = Kf <= 5 ? pick(std::integral_constant<int, 5>{})
                               : (Kf <= 9 ? pick(std::integral_constant<int, 9>{}) : pick(std::integral_constant<int, 25>{}));
            set_lds((const void *)fr, W * per);
            launch_timed("rap", l, fr, dim3(nblk(Nc, W)), dim3(64 * W), W * per, s, a, tb, F.A->coef.p, F.A->st.K,
                         F.A->st.doff.p, F.A->st.R, V.own.coef.p, Kc, V.own.st.doff.p, F.rap_R, F.rap_wx, F.rap_wy);
            KCHECK();
        } else if (l > 0) {
            Level &F = *lev[l - 1];
            XferArgs a = xfer_args(F, V, nullptr);
            const int Kc = V.own.st.K;
            const int S = 2 * F.rap_R + 1;
            // as many coarse cells (wavefronts) per workgroup as LDS allows
            auto lds_for = [&](int w) { return (size_t)64 * w * Kc * sizeof(double) + sizeof(int) * S * S * S; };
            const int W = lds_for(4) <= (size_t)lds_bytes ? 4 : (lds_for(2) <= (size_t)lds_bytes ? 2 : 1);
            if (lds_for(W) > (size_t)lds_bytes) fail(NKS_EINVAL, "coarse stencil of %d points exceeds the LDS", Kc);
            void (*fr)(XferArgs, const double *, int, const int8_t *, double *, int, const int *, int) =
                W == 4 ? k_rap<4> : (W == 2 ? k_rap<2> : k_rap<1>);
            set_lds((const void *)fr, lds_for(W));
            launch_timed("rap", l, fr, dim3(nblk(V.spp->N, W)), dim3(64 * W), lds_for(W), s, a, F.A->coef.p,
                         F.A->st.K, F.A->st.doff.p, V.own.coef.p, Kc, F.rap_slot.p, F.rap_R);
            KCHECK();
        }
        if (!ilu) continue;
        const TileDims &td = tiles_[l];
        FacArgs fa;
        fa.sub = V.sub.p;
        fa.blk = V.spp->blk.p;
        fa.lvlptr = V.lvlptr.p;
        fa.loc = V.loc.p;
        fa.inv = V.inv.p;
        fa.lexi = V.lexi.p;
        fa.upd_ptr = V.upd_ptr.p;
        fa.upd_k2 = V.upd_k2.p;
        fa.upd_t = V.upd_t.p;
        fa.lin = V.lin_pad.p;
        fa.A = V.A->coef.p;
        fa.N = V.spp->N;
        fa.NE = V.next_total;
        fa.amap = V.amap.p;
        fa.K = V.fst.K;
        fa.diag = V.fst.diag;
        fa.PX = td.PX;
        fa.PY = td.PY;
        fa.R = td.R;
        fa.Rz = td.Rz;
        fa.off = V.fst.doff.p;
        fa.w = V.w64.p;
        fa.err = V.err.p;
        const int *perm = (V.rows2d || use_rows3d(*this, V)) ? V.lexg.p : nullptr;
        bool stored = false;
        const int rl = V.box == 0 ? RowStencil<0>::NS + 2 : (V.box == 1 ? RowStencil<1>::NS + 2 : RowStencil<2>::NS + 2);
        const size_t sh_rows = sizeof(double) * (size_t)rl * V.max_next;
        if (V.rows2d && sh_rows <= (size_t)lds_bytes) {
            // 2D box in LDS, factored on the sweeps' wavefront schedule;
            // factors come out in lexicographic order
            IluRowsArgs ia{V.sub.p, V.spp->blk.p, V.slotmap.p, V.amap.p, V.A->coef.p, V.spp->N, V.next_total,
                           V.fst.diag, nullptr, nullptr, V.err.p};
            auto pick = [&](auto ft, auto dt) -> void (*)(IluRowsArgs) {
                using FT = decltype(ft);
                using DT = decltype(dt);
                return V.box == 0 ? k_ilu_rows<0, FT, DT>
                                  : (V.box == 1 ? k_ilu_rows<1, FT, DT> : k_ilu_rows<2, FT, DT>);
            };
            void (*fr)(IluRowsArgs) = nullptr;
            if (d.precision == NKS_FP64) {
                fr = pick(double{}, double{});
                ia.f = V.f64.p;
                ia.invd = V.invd64.p;
            } else if (d.precision == NKS_FP32) {
                fr = pick(float{}, float{});
                ia.f = V.f32.p;
                ia.invd = V.invd32.p;
            } else {
                fr = pick(uint16_t{}, float{});
                ia.f = V.f16.p;
                ia.invd = V.invd32.p;
            }
            set_lds((const void *)fr, sh_rows);
            // one wavefront eliminates; the box stencils' elimination holds
            // about 230 registers, so their workgroups are that one wavefront
            // alone (two rounds of the batch's coarse boxes instead of five)
            launch_timed("ilu_factor", l, fr, dim3(V.nsub), dim3(V.box == 0 ? 256 : 64), sh_rows, s, ia);
            KCHECK();
            stored = true;
        } else {
        const size_t sh_lds = sizeof(double) * (size_t)fa.K * V.max_next +
                              sizeof(int) * ((size_t)V.max_tile + V.max_nlev + 1 + 2 * (size_t)fa.K + 1 +
                                             2 * (size_t)V.nupd + V.max_next);
        void (*flds)(FacArgs, int, int, int) = nullptr;
        if (fa.diag <= 2 && V.max_upd <= 1) flds = k_ilu_factor_lds<2, 1>;
        else if (fa.diag <= 3 && V.max_upd <= 3) flds = k_ilu_factor_lds<3, 3>;
        else if (fa.diag <= 12 && V.max_upd <= 12) flds = k_ilu_factor_lds<12, 12>;
        if (flds && sh_lds <= (size_t)lds_bytes) {
            // the whole box fits in LDS (2D): fill and eliminate there
            set_lds((const void *)flds, sh_lds);
            // enough rows in flight for the widest hyperplane and for staging the box
            const int bsl = V.max_lvl <= 64 && V.max_next <= 512 ? 64 : 256;
            launch_timed("ilu_factor", l, flds, dim3(V.nsub), dim3(bsl), sh_lds, s, fa, V.max_next, V.max_tile,
                         V.nupd);
            KCHECK();
        } else {
            k_ilu_fill<<<V.nsub, 256, 0, s>>>(fa);
            KCHECK();
            // enough rows in flight for the widest hyperplane, up to 256
            const int bsg = V.max_lvl <= 64 ? 64 : (V.max_lvl <= 128 ? 128 : 256);
            const size_t sh = (size_t)bsg * fa.K * sizeof(double) + sizeof(int) * (size_t)(V.max_nlev + 1);
            set_lds((const void *)k_ilu_factor, sh);
            launch_timed("ilu_factor", l, k_ilu_factor, dim3(V.nsub), dim3(bsg), sh, s, fa);
            KCHECK();
        }
        }
        const int NE = V.next_total;
        if (stored) {
            // the row factorisation wrote the storage precision itself
        } else if (d.precision == NKS_FP64) {
            k_ilu_store<double, double><<<nblk(NE, 256), 256, 0, s>>>(V.w64.p, NE, fa.K, fa.diag, V.f64.p, V.invd64.p, perm);
        } else if (d.precision == NKS_FP32) {
            k_ilu_store<float, float><<<nblk(NE, 256), 256, 0, s>>>(V.w64.p, NE, fa.K, fa.diag, V.f32.p, V.invd32.p, perm);
        } else {
            k_ilu_store<uint16_t, float><<<nblk(NE, 256), 256, 0, s>>>(V.w64.p, NE, fa.K, fa.diag, V.f16.p, V.invd32.p, perm);
        }
        KCHECK();
        if (l == L - 1 && cp.on) pack_runs();
    }
}

Ras::~Ras() {
    if (hpiv) (void)hipHostFree(hpiv);
}

void Ras::check_pivots() {
    if (!hpiv) HIPC(hipHostMalloc((void **)&hpiv, sizeof(int) * 8));
    for (int l = 0; l < L; ++l)
        HIPC(hipMemcpyAsync(hpiv + l, lev[l]->err.p, sizeof(int), hipMemcpyDeviceToHost, g->s));
    HIPC(hipStreamSynchronize(g->s));
    count_host_wait();
    for (int l = 0; l < L; ++l)
        if (hpiv[l]) {
            const int bits = hpiv[l];
            HIPC(hipMemsetAsync(lev[l]->err.p, 0, sizeof(int), g->s));
            if (bits & 1) fail(NKS_EZEROPIVOT, "zero pivot in a subdomain ILU(0) factorization on level %d", l);
            fail(NKS_EHIP, "a 3D subdomain sweep on level %d gave up waiting for its neighbouring slab", l);
        }
}

static int level_index(const Ras &M, const Level &V) {
    for (int l = 0; l < M.L; ++l)
        if (M.lev[l].get() == &V) return l;
    return -1;
}

// workgroups of a kernel that fit on one CU at once (registers and LDS),
// cached per kernel and LDS size
static int rows_occupancy(const void *fn, int threads, size_t sh) {
    static std::mutex mu;
    static std::map<std::pair<const void *, size_t>, int> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({fn, sh});
    if (it != cache.end()) return it->second;
    set_lds(fn, sh);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, sh) != hipSuccess) {
        (void)hipGetLastError();
        nb = 1;
    }
    cache[{fn, sh}] = std::max(nb, 1);
    return std::max(nb, 1);
}

// AS / right-RAS: sum the boxes' extended values into z (left-RAS writes
// the owned cells in the sweep)
static void gather_ext(Ras &M, Level &V, double *z, const int *mask, bool accumulate) {
    if (M.d.variant == NKS_LEFT_RAS) return;
    k_ras_gather<<<nblk(V.spp->N, 256), 256, 0, M.g->s>>>(V.spp->blk.p, V.spp->B, V.spp->N, V.part.p, V.sub.p,
                                                          V.zext.p, z, mask, accumulate ? 1 : 0);
    KCHECK();
}

template <typename FT, typename VT, typename DT>
static void launch_rows(Ras &M, Level &V, const double *r, double *z, const int *mask, bool accumulate) {
    RowsArgs a{};
    a.sub = V.sub.p;
    if (V.box == 0) row_kmap<0, FT>(V.hslot, a.kmap);
    else if (V.box == 1) row_kmap<1, FT>(V.hslot, a.kmap);
    else row_kmap<2, FT>(V.hslot, a.kmap);
    if (M.d.precision == NKS_FP64) a.F = V.f64.p;
    else if (M.d.precision == NKS_FP32) a.F = V.f32.p;
    else a.F = V.f16.p;
    a.invd = M.d.precision == NKS_FP64 ? (const void *)V.invd64.p : (const void *)V.invd32.p;
    a.NE = V.next_total;
    a.r = r;
    a.z = z;
    a.zext = V.zext.p;
    a.mask = mask;
    a.variant = M.d.variant;
    a.accumulate = accumulate ? 1 : 0;
    // LDS strides: both runs of a cell side by side (four wavefronts), or one
    // run at a time (one wavefront)
    const int CS4 = V.box == 0 ? row_stride<0, FT>() : (V.box == 1 ? row_stride<1, FT>() : row_stride<2, FT>());
    const int CS1 = V.box == 0 ? row_half_stride<0, FT>()
                               : (V.box == 1 ? row_half_stride<1, FT>() : row_half_stride<2, FT>());
    const size_t n = V.max_next;
    const size_t sh4 = rows_lds(sizeof(VT), sizeof(FT), sizeof(DT), CS4, rows_pad(V.box), n).total;
    const size_t sh1 = rows_lds(sizeof(VT), sizeof(FT), sizeof(DT), CS1, rows_pad(V.box), n).total;
    if (V.max_next >= (1 << 16)) fail(NKS_EINVAL, "2D subdomain of %zu cells exceeds 65535", n);
    if (sh4 > (size_t)M.lds_bytes) fail(NKS_EINVAL, "2D subdomain of %zu cells does not fit in LDS", n);
    void (*fn4)(RowsArgs) = V.box == 0 ? k_ras_rows<FT, VT, DT, 0, 256>
                                       : (V.box == 1 ? k_ras_rows<FT, VT, DT, 1, 256> : k_ras_rows<FT, VT, DT, 2, 256>);
    void (*fn1)(RowsArgs) = V.box == 0 ? k_ras_rows<FT, VT, DT, 0, 64>
                                       : (V.box == 1 ? k_ras_rows<FT, VT, DT, 1, 64> : k_ras_rows<FT, VT, DT, 2, 64>);
    // One-wavefront workgroups when, holding both runs, they would let at
    // least twice as many boxes sweep at once on a CU (the four-wavefront
    // form is bound by its idle staging wavefronts' registers) and the launch
    // has the boxes to use it: small boxes, whose staging is short.  Large
    // boxes keep the four-wavefront form, which stages the upper runs during
    // the forward sweep (measured on MI355X: 36 x 36 boxes sweep 20% slower
    // with one wavefront).  The one-wavefront form then holds one run at a
    // time, which lets more of its boxes sweep at once.
    const int occ4 = rows_occupancy((const void *)fn4, 256, sh4), occ1 = rows_occupancy((const void *)fn1, 64, sh4);
    const bool one = occ1 >= 2 * occ4 && V.nsub > M.n_cu * occ4;
    const int occ = one ? rows_occupancy((const void *)fn1, 64, sh1) : occ4;
    void (*fnp)(PackArgs) = V.box == 0 ? k_ras_packed<FT, VT, DT, 0>
                                       : (V.box == 1 ? k_ras_packed<FT, VT, DT, 1> : k_ras_packed<FT, VT, DT, 2>);
    const size_t shp = packed_lds(sizeof(VT), sizeof(FT), sizeof(DT), CS4, V.box, V.pk_max_n).total;
    // A packed group sweeps about as long as one of its boxes (the sweep is
    // bound by its step latency, measured on MI355X), so groups pay off when
    // they take fewer rounds of workgroups over the CUs than single boxes.
    auto rounds = [&](int wgs, int per_cu) { return (wgs + M.n_cu * per_cu - 1) / (M.n_cu * per_cu); };
    if (V.pk_groups > 0 && rounds(V.pk_groups, rows_occupancy((const void *)fnp, 256, shp)) <= rounds(V.nsub, occ)) {
        // small boxes: groups of them packed into one sweeping wavefront
        PackArgs p{};
        p.sub = V.sub.p;
        p.glane = V.pk_lane.p;
        p.gsteps = V.pk_steps.p;
        p.gbox = V.pk_box.p;
        p.ext2glob = V.pk_e2g.p;
        p.F = a.F;
        p.invd = a.invd;
        p.NE = a.NE;
        p.r = r;
        p.z = z;
        p.zext = a.zext;
        p.mask = mask;
        p.variant = a.variant;
        p.accumulate = a.accumulate;
        for (int q = 0; q < 32; ++q) p.kmap[q] = a.kmap[q];
        set_lds((const void *)fnp, shp);
        V.form = NKS_SWEEP_PACKED;
        V.form_wgs = V.pk_groups;
        launch_sweep("ras_apply", level_index(M, V), fnp, dim3(V.pk_groups), dim3(256), shp, M.g->s, p);
        KCHECK();
        gather_ext(M, V, z, mask, accumulate);
        return;
    }
    void (*fn)(RowsArgs) = one ? fn1 : fn4;
    const size_t sh = one ? sh1 : sh4;
    set_lds((const void *)fn, sh);
    V.form = one ? NKS_SWEEP_ROWS1 : NKS_SWEEP_ROWS4;
    V.form_wgs = V.nsub;
    launch_sweep("ras_apply", level_index(M, V), fn, dim3(V.nsub), dim3(one ? 64 : 256), sh, M.g->s, a);
    KCHECK();
    gather_ext(M, V, z, mask, accumulate);
}

// LDS of the 3D row sweep for boxes of n cells: rv[n + 1], the
// padded lower and upper runs, 1/u_ii
static size_t rows3d_lds(int precision, size_t n, bool half = false) {
    const size_t ft = precision == NKS_FP64 ? 8 : (precision == NKS_FP32 ? 4 : 2);
    const size_t vt = precision == NKS_FP64 ? 8 : 4, dt = vt;
    const size_t nlp = precision == NKS_FP64 ? rows3d_lpad<double>()
                                             : (precision == NKS_FP32 ? rows3d_lpad<float>() : rows3d_lpad<uint16_t>());
    return al16(vt * (n + 1)) + al16(ft * (half ? 1 : 2) * nlp * n) + al16(dt * n);
}

// whether a level runs the 3D row sweep (its factors are then
// stored in lexicographic order)
static bool use_rows3d(const Ras &M, const Level &V) {
    return V.rows3d && V.max_next < (1 << 16) && rows3d_lds(M.d.precision, V.max_next, true) <= (size_t)M.lds_bytes;
}

template <typename FT, typename VT, typename DT>
static void launch_rows3d(Ras &M, Level &V, const double *r, double *z, const int *mask, bool accumulate) {
    Rows3Args a{};
    a.sub = V.sub.p;
    constexpr int NLP = rows3d_lpad<FT>();
    static_assert(2 * NLP <= 16, "run map fits the argument block");
    for (int q = 0; q < 16; ++q) a.kmap[q] = -1;
    for (int q = 0; q < 3; ++q) {
        a.kmap[q] = V.hkmap3[q];
        a.kmap[NLP + q] = V.hkmap3[3 + q];
    }
    if (M.d.precision == NKS_FP64) a.F = V.f64.p;
    else if (M.d.precision == NKS_FP32) a.F = V.f32.p;
    else a.F = V.f16.p;
    a.invd = M.d.precision == NKS_FP64 ? (const void *)V.invd64.p : (const void *)V.invd32.p;
    a.NE = V.next_total;
    a.r = r;
    a.z = z;
    a.zext = V.zext.p;
    a.mask = mask;
    a.err = V.err.p;
    a.variant = M.d.variant;
    a.accumulate = accumulate ? 1 : 0;
    // a wavefront per slab: four per workgroup, or eight for boxes of five
    // to eight slabs; both runs of every cell in LDS, or one at a time where
    // both do not fit
    const bool half = rows3d_lds(M.d.precision, V.max_next) > (size_t)M.lds_bytes;
    const size_t sh = rows3d_lds(M.d.precision, V.max_next, half);
    const bool eight = V.rows3d_multi && V.rows3d_slabs > 4;
    void (*fn)(Rows3Args) =
        !V.rows3d_multi ? (half ? k_ras_rows3d<FT, VT, DT, false, 256, true> : k_ras_rows3d<FT, VT, DT, false, 256, false>)
        : eight ? (half ? k_ras_rows3d<FT, VT, DT, true, 512, true> : k_ras_rows3d<FT, VT, DT, true, 512, false>)
                : (half ? k_ras_rows3d<FT, VT, DT, true, 256, true> : k_ras_rows3d<FT, VT, DT, true, 256, false>);
    set_lds((const void *)fn, sh);
    V.form = NKS_SWEEP_ROWS3D;
    V.form_wgs = V.nsub;
    launch_sweep("ras_apply", level_index(M, V), fn, dim3(V.nsub), dim3(eight ? 512 : 256), sh, M.g->s, a);
    KCHECK();
    gather_ext(M, V, z, mask, accumulate);
}

template <typename FT, typename VT, typename DT>
static void launch_apply(Ras &M, Level &V, const TileDims &td, const double *r, double *z, const int *mask,
                         bool accumulate) {
    if (V.rows2d) {
        launch_rows<FT, VT, DT>(M, V, r, z, mask, accumulate);
        return;
    }
    if (use_rows3d(M, V)) {
        launch_rows3d<FT, VT, DT>(M, V, r, z, mask, accumulate);
        return;
    }
    ApplyArgs a;
    a.sub = V.sub.p;
    a.blk = V.spp->blk.p;
    a.lvlptr = V.lvlptr.p;
    a.loc = V.loc.p;
    a.lexi = V.lexi.p;
    a.lin = V.lin_pad.p;
    if (M.d.precision == NKS_FP64) a.F = V.f64.p;
    else if (M.d.precision == NKS_FP32) a.F = V.f32.p;
    else a.F = V.f16.p;
    a.invd = M.d.precision == NKS_FP64 ? (const void *)V.invd64.p : (const void *)V.invd32.p;
    a.NE = V.next_total;
    a.K = V.fst.K;
    a.diag = V.fst.diag;
    a.PX = td.PX;
    a.PY = td.PY;
    a.PZ = td.PZ;
    a.R = td.R;
    a.Rz = td.Rz;
    a.tile = td.PX * td.PY * td.PZ;
    a.r = r;
    a.z = z;
    a.zext = V.zext.p;
    a.mask = mask;
    a.variant = M.d.variant;
    a.accumulate = accumulate ? 1 : 0;
    const int ncmax = std::max(a.diag, a.K - a.diag - 1);
    const size_t budget = (size_t)M.lds_bytes;
    a.maxlev = V.max_nlev;
    const size_t fixed = apply_lds(sizeof(VT), sizeof(FT), sizeof(DT), a.tile, ncmax, 0, a.maxlev).total + 64;
    const size_t per = sizeof(FT) * (size_t)ncmax + sizeof(DT) + sizeof(int);
    if (fixed + per * (size_t)V.max_lvl > budget)
        fail(NKS_EINVAL, "subdomain tile of %d cells and hyperplanes of %d cells do not fit in LDS (%zu bytes)",
             a.tile, V.max_lvl, budget);
    a.cap = (int)std::min<size_t>((budget - fixed) / per, (size_t)V.max_next);
    a.cap = std::max(a.cap, V.max_lvl);
    const size_t sh = apply_lds(sizeof(VT), sizeof(FT), sizeof(DT), a.tile, ncmax, a.cap, a.maxlev).total;
    if (sh > budget) fail(NKS_EINVAL, "LDS layout of %zu bytes exceeds %zu", sh, budget);
    const bool seven = a.K == 7 && a.diag == 3;
    if (seven)
        for (int k = 0; k < 7; ++k) {
            const int8_t *o = &V.fst.off[3 * k];
            a.lin7[k] = o[0] + td.PX * (o[1] + td.PY * o[2]);
        }
    const void *fn = seven ? (const void *)k_ras_apply<FT, VT, DT, 3> : (const void *)k_ras_apply<FT, VT, DT, 0>;
    set_lds(fn, sh);
    // enough threads for the widest hyperplane: small boxes with wide
    // stencils have many short hyperplanes, where one wavefront's barriers
    // are the cheap ones
    const int bs = V.max_lvl <= 64 ? 64 : (V.max_lvl <= 128 ? 128 : 256);
    V.form = NKS_SWEEP_HYPERPLANE;
    V.form_wgs = V.nsub;
    {
        if (seven)
            launch_sweep("ras_apply", level_index(M, V), k_ras_apply<FT, VT, DT, 3>, dim3(V.nsub), dim3(bs), sh, M.g->s, a);
        else
            launch_sweep("ras_apply", level_index(M, V), k_ras_apply<FT, VT, DT, 0>, dim3(V.nsub), dim3(bs), sh, M.g->s, a);
        KCHECK();
    }
    gather_ext(M, V, z, mask, accumulate);
}

void Ras::apply_level(int l, const double *r, double *z, const int *mask, bool accumulate) {
    Level &V = *lev[l];
    const TileDims &td = tiles_[l];
    if (d.precision == NKS_FP64) launch_apply<double, double, double>(*this, V, td, r, z, mask, accumulate);
    else if (d.precision == NKS_FP32) launch_apply<float, float, float>(*this, V, td, r, z, mask, accumulate);
    else launch_apply<uint16_t, float, float>(*this, V, td, r, z, mask, accumulate);
}

void Ras::restrict_to(int l, const double *rf, double *rc, const int *mask) {
    XferArgs a = xfer_args(*lev[l], *lev[l + 1], mask);
    const Space &C = *lev[l + 1]->spp;
    if (a.cs[0] <= 8) k_restrict<8><<<(int)C.htile.size(), TILE, 0, g->s>>>(a, C.tile.p, rf, rc);
    else k_restrict<16><<<(int)C.htile.size(), TILE, 0, g->s>>>(a, C.tile.p, rf, rc);
    KCHECK();
}

void Ras::prolong_add(int l, const double *ec, double *zf, const int *mask) {
    XferArgs a = xfer_args(*lev[l], *lev[l + 1], mask);
    const Space &F = *lev[l]->spp;
    k_prolong_add<<<(int)F.htile.size(), TILE, 0, g->s>>>(a, F.tile.p, ec, zf);
    KCHECK();
}

// ---------------------------------------------------------------- persistent coarse solve (host)
// Whether the coarsest level's GMRES runs as one persistent launch, and its
// tables: per reservoir its boxes packed into lane groups (a box's rows on
// consecutive lanes of one wavefront, a new group when the next box's rows
// no longer fit), the map from every extended cell to the reservoir cell it
// copies and from every cell to the extended cell of the box that owns it.

void Ras::setup_persistent() {
    cp.on = false;
    if (L < 2 || d.coarse_kernel == NKS_COARSE_CHUNKED) return;
    Level &C = *lev[L - 1];
    const Space &S = *C.spp;
    const bool need = d.coarse_kernel == NKS_COARSE_PERSISTENT;
    auto refuse = [&](const char *why) {
        if (need) fail(NKS_EINVAL, "persistent coarse solve: %s", why);
    };
    if (!C.rows2d) return refuse("the coarsest level is not a 2D level swept by rows");
    if (d.variant != NKS_LEFT_RAS) return refuse("it runs the left-RAS variant only");
    if (C.A->st.K > 25) return refuse("coarse stencil wider than 5x5");
    int ncap = 0;
    for (int b = 0; b < S.B; ++b) {
        if (S.hblk[b].nz != 1) return refuse("the coarsest level is not 2D");
        ncap = std::max(ncap, S.hblk[b].nx * S.hblk[b].ny);
    }
    if (ncap > COARSE_CELLS) return refuse("more than 4096 cells per reservoir on the coarsest level");
    const int LB = C.box == 0 ? RowStencil<0>::LB : (C.box == 1 ? RowStencil<1>::LB : RowStencil<2>::LB);
    std::vector<int> efirst(S.B + 1, 0), gfirst(S.B + 1, 0), gsteps, ext2loc(C.next_total, -1),
        own2ext(S.N, -1);
    std::vector<int2> glane;
    int max_ne = 0;
    for (int b = 0; b < S.B; ++b) {
        const Blk &k = S.hblk[b];
        const BlkPart &pt = C.hpart[b];
        const int nbox = pt.px * pt.py * pt.pz;
        const SubDev &last = C.hsub[pt.first + nbox - 1];
        efirst[b] = C.hsub[pt.first].fac_off;
        max_ne = std::max(max_ne, last.fac_off + last.next - efirst[b]);
        gfirst[b] = (int)gsteps.size();
        int used = 64;
        for (int q = pt.first; q < pt.first + nbox; ++q) {
            const SubDev &sd = C.hsub[q];
            if (sd.ey > 64) return refuse("a coarse box of more than 64 rows");
            if (used + sd.ey > 64) {
                glane.resize(glane.size() + 64, int2{q, -1});
                gsteps.push_back(0);
                used = 0;
            }
            const size_t gq = gsteps.size() - 1;
            for (int y = 0; y < sd.ey; ++y) glane[gq * 64 + used + y] = int2{q, y};
            used += sd.ey;
            gsteps[gq] = std::max(gsteps[gq], (sd.ex - 1) + LB * (sd.ey - 1) + 1);
            for (int y = 0; y < sd.ey; ++y)
                for (int x = 0; x < sd.ex; ++x) {
                    const int loc = (sd.gorg - k.off) + x + k.nx * y;
                    ext2loc[sd.fac_off + x + sd.ex * y] = loc;
                    if (x >= sd.lx0 && x < sd.lx1 && y >= sd.ly0 && y < sd.ly1) {
                        if (own2ext[k.off + loc] >= 0) fail(NKS_EINVAL, "coarse cell owned twice");
                        own2ext[k.off + loc] = sd.fac_off + x + sd.ex * y;
                    }
                }
        }
    }
    efirst[S.B] = C.next_total;
    gfirst[S.B] = (int)gsteps.size();
    for (int i = 0; i < S.N; ++i)
        if (own2ext[i] < 0) fail(NKS_EINVAL, "coarse cell %d owned by no box", i);
    const int m = coarse.m;
    const size_t vt = d.precision == NKS_FP64 ? 8 : 4;
    const int nw = (d.precision == NKS_FP64 ? 512 : 1024) / 64;
    const size_t lds = sizeof(double) * (2 * (size_t)ncap + 40 + (size_t)m * m + 4 * m + 1 + 8 * nw) +
                       4 * sizeof(int) + vt * ((size_t)max_ne + 1);
    if (lds > (size_t)lds_bytes) return refuse("the largest reservoir's boxes do not fit in LDS");
    // One workgroup streams its reservoir's factor runs through one CU in
    // every sweep; measured on MI355X, that outruns the chunked launches only
    // while they stay small (a 64 x 64 coarse level of 12 x 12 boxes, 0.9 MB
    // of FP32 runs, sweeps at about 1.4 us per wavefront step).  The
    // automatic choice takes the persistent form up to 256 KiB of runs.
    const size_t run_bytes =
        d.precision == NKS_FP64
            ? (C.box == 0 ? row_run<0, double>() : (C.box == 1 ? row_run<1, double>() : row_run<2, double>())) * 8
            : (d.precision == NKS_FP32
                   ? (C.box == 0 ? row_run<0, float>() : (C.box == 1 ? row_run<1, float>() : row_run<2, float>())) * 4
                   : (C.box == 0 ? row_run<0, uint16_t>()
                                 : (C.box == 1 ? row_run<1, uint16_t>() : row_run<2, uint16_t>())) * 2);
    if (!need && (size_t)max_ne * run_bytes > COARSE_AUTO_RUN_BYTES) return;
    hipStream_t s = g->s;
    cp.ncap = ncap;
    cp.max_ne = max_ne;
    cp.lds = lds;
    cp.efirst.upload(&g->al, efirst, s);
    cp.gfirst.upload(&g->al, gfirst, s);
    cp.gsteps.upload(&g->al, gsteps, s);
    cp.glane.upload(&g->al, glane, s);
    cp.ext2loc.upload(&g->al, ext2loc, s);
    cp.own2ext.upload(&g->al, own2ext, s);
    // the padded runs depend on the factor type
    int km[32];
    std::vector<int> kv(32);
    const int NE = C.next_total;
    if (d.precision == NKS_FP64) {
        if (C.box == 0) row_kmap<0, double>(C.hslot, km);
        else if (C.box == 1) row_kmap<1, double>(C.hslot, km);
        else row_kmap<2, double>(C.hslot, km);
        const int run = C.box == 0 ? row_run<0, double>() : (C.box == 1 ? row_run<1, double>() : row_run<2, double>());
        cp.r64.alloc(&g->al, (size_t)NE * run);
    } else if (d.precision == NKS_FP32) {
        if (C.box == 0) row_kmap<0, float>(C.hslot, km);
        else if (C.box == 1) row_kmap<1, float>(C.hslot, km);
        else row_kmap<2, float>(C.hslot, km);
        const int run = C.box == 0 ? row_run<0, float>() : (C.box == 1 ? row_run<1, float>() : row_run<2, float>());
        cp.r32.alloc(&g->al, (size_t)NE * run);
    } else {
        if (C.box == 0) row_kmap<0, uint16_t>(C.hslot, km);
        else if (C.box == 1) row_kmap<1, uint16_t>(C.hslot, km);
        else row_kmap<2, uint16_t>(C.hslot, km);
        const int run =
            C.box == 0 ? row_run<0, uint16_t>() : (C.box == 1 ? row_run<1, uint16_t>() : row_run<2, uint16_t>());
        cp.r16.alloc(&g->al, (size_t)NE * run);
    }
    for (int q = 0; q < 32; ++q) kv[q] = km[q];
    cp.kmap.upload(&g->al, kv, s);
    cp.V.alloc(&g->al, (size_t)(m + 1) * S.N);
    cp.its.alloc(&g->al, S.B);
    cp.res.alloc(&g->al, S.B);
    cp.on = true;
}

template <typename FT, int BOX>
static void pack_runs_t(Ras &M, Level &C, const FT *F, FT *runs) {
    constexpr int RUN = row_run<BOX, FT>();
    k_pack_runs<FT, RUN><<<nblk(C.next_total, 256), 256, 0, M.g->s>>>(F, C.next_total, M.cp.kmap.p, runs);
    KCHECK();
}

void Ras::pack_runs() {
    Level &C = *lev[L - 1];
    if (d.precision == NKS_FP64) {
        if (C.box == 0) pack_runs_t<double, 0>(*this, C, C.f64.p, cp.r64.p);
        else if (C.box == 1) pack_runs_t<double, 1>(*this, C, C.f64.p, cp.r64.p);
        else pack_runs_t<double, 2>(*this, C, C.f64.p, cp.r64.p);
    } else if (d.precision == NKS_FP32) {
        if (C.box == 0) pack_runs_t<float, 0>(*this, C, C.f32.p, cp.r32.p);
        else if (C.box == 1) pack_runs_t<float, 1>(*this, C, C.f32.p, cp.r32.p);
        else pack_runs_t<float, 2>(*this, C, C.f32.p, cp.r32.p);
    } else {
        if (C.box == 0) pack_runs_t<uint16_t, 0>(*this, C, C.f16.p, cp.r16.p);
        else if (C.box == 1) pack_runs_t<uint16_t, 1>(*this, C, C.f16.p, cp.r16.p);
        else pack_runs_t<uint16_t, 2>(*this, C, C.f16.p, cp.r16.p);
    }
}

template <typename FT, typename VT, typename DT>
static void launch_coarse(Ras &M, Level &C, CoarseArgs &a) {
    // 1024 threads (four wavefronts per SIMD, 128 registers each) for the
    // FP32 sweeps, 512 for the FP64 ones, whose runs take twice the registers
    constexpr int NT = sizeof(VT) == 8 ? 512 : 1024;
    void (*fn)(CoarseArgs) = C.box == 0 ? k_coarse_gmres<FT, VT, DT, 0, NT>
                                        : (C.box == 1 ? k_coarse_gmres<FT, VT, DT, 1, NT> : k_coarse_gmres<FT, VT, DT, 2, NT>);
    set_lds((const void *)fn, M.cp.lds);
    launch_timed("coarse_gmres", M.L - 1, fn, dim3(C.spp->B), dim3(NT), M.cp.lds, M.g->s, a);
    KCHECK();
}

void Ras::coarse_persistent(const double *b, double *x, const int *mask) {
    Level &C = *lev[L - 1];
    const Op &A = *C.A;
    CoarseArgs a{};
    a.blk = C.spp->blk.p;
    a.sub = C.sub.p;
    a.efirst = cp.efirst.p;
    a.gfirst = cp.gfirst.p;
    a.glane = cp.glane.p;
    a.gsteps = cp.gsteps.p;
    a.ext2loc = cp.ext2loc.p;
    a.own2ext = cp.own2ext.p;
    a.invd = d.precision == NKS_FP64 ? (const void *)C.invd64.p : (const void *)C.invd32.p;
    a.runs = d.precision == NKS_FP64 ? (const void *)cp.r64.p
                                     : (d.precision == NKS_FP32 ? (const void *)cp.r32.p : (const void *)cp.r16.p);
    a.coef = A.coef.p;
    a.K = A.st.K;
    a.N = C.spp->N;
    for (int q = 0; q < 25; ++q) {
        const int qq = std::min(q, A.st.K - 1);
        a.offp[q] = (A.st.off[3 * qq] & 0xff) | ((A.st.off[3 * qq + 1] & 0xff) << 8);
    }
    a.b = b;
    a.x = x;
    a.V = cp.V.p;
    a.mask = mask;
    a.its = cp.its.p;
    a.res = cp.res.p;
    a.m = coarse.m;
    a.maxit = d.coarse_maxit;
    a.rtol = d.coarse_rtol;
    a.atol = 0.0;
    a.ncap = cp.ncap;
    if (d.precision == NKS_FP64) launch_coarse<double, double, double>(*this, C, a);
    else if (d.precision == NKS_FP32) launch_coarse<float, float, float>(*this, C, a);
    else launch_coarse<uint16_t, float, float>(*this, C, a);
}

static void zero(const Space &S, double *x, hipStream_t s) {
    k_fill<<<nblk(S.N, 256), 256, 0, s>>>(S.N, 0.0, x);
    KCHECK();
}

void Ras::coarse_solve(const double *b, double *x, const int *mask) {
    if (cp.on) {
        coarse_persistent(b, x, mask);
        ++coarse_calls;
        return;
    }
    Level &C = *lev[L - 1];
    const Space &S = *C.spp;
    hipStream_t s = g->s;
    zero(S, x, s);
    MatVec A = [&](const double *xx, double *yy, const double *bb, const int *mk) {
        launch_spmv(*C.A, xx, yy, bb, mk, s);
    };
    Precond P = [&](const double *rr, double *zz, const int *mk) { apply_level(L - 1, rr, zz, mk, false); };
    GmOpts o;
    o.rtol = d.coarse_rtol;
    o.atol = 0.0;
    o.maxit = d.coarse_maxit;
    // the preconditioned basis z_j = M v_j is kept, so a cycle ends with
    // x0 + Z y (the iterate x0 + M V y of right preconditioning, by the
    // linearity of the fixed M) instead of a combination, one more sweep and
    // an update
    o.flexible = true;
    o.check_every = 1;
    o.graph_chunk = graph_chunk;
    // one Gram-Schmidt pass: a handful of iterations to a loose tolerance
    o.single_pass = true;
    coarse.solve(A, P, b, x, true, o, mask, s, C.A);
    ++coarse_calls;
}

// X = MG(b, l, 0) (Algorithm 1) in the composition selected by the cycle type
void Ras::vcycle(int l, const double *b, double *x, const int *mask) {
    if (l == L - 1) {
        coarse_solve(b, x, mask);
        return;
    }
    Level &F = *lev[l];
    Level &C = *lev[l + 1];
    const Space &S = *F.spp;
    hipStream_t s = g->s;
    const int cyc = d.cycle;
    if (cyc == NKS_ADDITIVE || cyc == NKS_COARSE_ONLY) {
        restrict_to(l, b, C.bc.p, mask);
        vcycle(l + 1, C.bc.p, C.xc.p, mask);
        zero(S, x, s);
        prolong_add(l, C.xc.p, x, mask);
        if (cyc == NKS_ADDITIVE) apply_level(l, b, x, mask, true);
        return;
    }
    int mu = d.mu, nu = d.nu;
    if (cyc == NKS_LEFT_KASKADE) { mu = 0; nu = 1; }
    if (cyc == NKS_RIGHT_KASKADE) { mu = 1; nu = 0; }
    const double *rr = b;
    if (mu == 0) {
        zero(S, x, s);
    } else {
        apply_level(l, b, x, mask, false);          // x = M^{-1} b (x started at 0)
        for (int k = 1; k < mu; ++k) {
            launch_spmv(*F.A, x, F.r.p, b, mask, s);
            apply_level(l, F.r.p, x, mask, true);
        }
        launch_spmv(*F.A, x, F.r.p, b, mask, s);
        rr = F.r.p;
    }
    restrict_to(l, rr, C.bc.p, mask);
    vcycle(l + 1, C.bc.p, C.xc.p, mask);
    prolong_add(l, C.xc.p, x, mask);
    for (int k = 0; k < nu; ++k) {
        launch_spmv(*F.A, x, F.r.p, b, mask, s);
        apply_level(l, F.r.p, x, mask, true);
    }
}

void Ras::apply(const double *r, double *z, const int *mask) {
    if (L == 1) apply_level(0, r, z, mask, false);
    else vcycle(0, r, z, mask);
}

}  // namespace nks
