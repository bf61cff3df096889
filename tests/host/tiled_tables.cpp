// Host check of the tiled sweep's tables (build_mj_table) for a stencil plan
// of the two-species cascade on an S1 x S2 grid: every state owned once,
// every list in bounds and consistent with the operator's columns, every
// ring position owned by a workgroup in the neighbour set, and an emulation
// of the kernel's rounds (the same data flow in double arithmetic, each LDS
// value tagged with the step it holds and every read checking the tag)
// against plain jumps of the whole vector, which it must equal exactly.
//
// usage: tiled_tables S1 S2 cap S [rounds]; exit 0 when every check holds.
#include "persistent.hip"

#include <cstdio>
#include <cstdlib>
#include <random>

using namespace mjp;

// the table builder needs neither device memory nor error text for stencil plans
mjp_status mjp::DevBuf::reserve(size_t) { return MJP_OK; }
void mjp::DevBuf::release() {}
mjp_status mjp::fail(mjp_status s, const char*, ...) { return s; }

int main(int argc, char** argv) {
    if (argc < 5) {
        std::fprintf(stderr, "usage: %s S1 S2 cap S [rounds]\n", argv[0]);
        return 2;
    }
    const int S1 = std::atoi(argv[1]), S2 = std::atoi(argv[2]), cap = std::atoi(argv[3]), S = std::atoi(argv[4]);
    const int rounds = argc > 5 ? std::atoi(argv[5]) : 3;
    if (S != 4 && S != 8) return 2;
    const int kLoad = mj_load_cap(S), kHalo = mj_halo_cap(S), kX = mj_x_cap(S);
    constexpr int W = 5;
    mjp_plan p;
    p.kind = PLAN_STENCIL;
    p.n = (int64_t)S1 * S2;
    p.coef.model = MJP_MODEL_CASCADE2;
    p.coef.S1 = S1;
    p.coef.S2 = S2;
    p.coef.leaky = 0;
    const float rates[6] = {0.01f, 0.003f, 0.002f, 0.004f, 0.f, 0.f};
    for (int j = 0; j < 6; ++j) p.coef.c[j] = rates[j];
    std::vector<int32_t> tab;
    int G = 0;
    if (!build_mj_table(&p, W, S, cap, tab, G)) {
        std::printf("table does not fit\n");
        return 1;
    }
    const int64_t n = p.n;
    auto hdr = [&](int g) { return tab.data() + (size_t)kMJHdr * g; };
    auto entries = [&](int64_t m, int32_t* cc, float* vv, float& lo) {
        int32_t c6[kStencilMaxW];
        float v6[kStencilMaxW];
        stencil_entries<kStencilMaxW>(p.coef, m, c6, v6, lo);
        for (int j = 0; j < W; ++j) {
            cc[j] = c6[j];
            vv[j] = v6[j];
        }
    };
    long bad = 0;
    auto check = [&](bool ok, const char* what, int g) {
        if (!ok && bad++ < 8) std::printf("workgroup %d: %s\n", g, what);
    };

    // every state owned exactly once
    std::vector<int32_t> owner(n, -1), place(n, -1);
    for (int g = 0; g < G; ++g) {
        const int32_t* hd = hdr(g);
        const int n0 = hd[0];
        check(n0 >= 0 && n0 <= kMJOwn, "own rows beyond the tile", g);
        const int32_t* gid = tab.data() + hd[kMJHOwn];
        for (int i = 0; i < n0; ++i) {
            const bool ok = gid[i] >= 0 && gid[i] < n && owner[gid[i]] < 0;
            check(ok, "own row out of range or owned twice", g);
            if (ok) {
                owner[gid[i]] = g;
                place[gid[i]] = i;
            }
        }
    }
    for (int64_t m = 0; m < n; ++m) check(owner[m] >= 0, "a state nobody owns", -1);

    // per workgroup: positions, local columns, ring structure
    for (int g = 0; g < G; ++g) {
        const int32_t* hd = hdr(g);
        int nS[9];
        for (int j = 0; j <= S; ++j) nS[j] = hd[j];
        const int n0 = nS[0], nh = nS[S - 1] - n0, nl = nS[S] - n0;
        check(nl <= kLoad && nh <= kHalo && nS[S] <= kX, "rings beyond the LDS capacity", g);
        const int32_t* og = tab.data() + hd[kMJHOwn];
        const int32_t* ol = og + n0;
        const int32_t* rg = tab.data() + hd[kMJHRing];
        const int32_t* rl = rg + nh;
        const int32_t* ps = tab.data() + hd[kMJHPos];
        std::vector<int64_t> L(nS[S], -1);  // local place -> state
        for (int i = 0; i < n0; ++i) L[i] = og[i];
        std::vector<char> seen(nl, 0);
        for (int h = 0; h < nl; ++h) {
            check(h == 0 || ps[h] > ps[h - 1], "ring positions not ascending", g);
            const int loc = ps[nl + h];
            if (loc < 0 || loc >= nl || seen[loc]++) {
                check(false, "ring place out of range or repeated", g);
                continue;
            }
            const int o = ps[h] / kMJOwn, li = ps[h] % kMJOwn;
            if (o < 0 || o >= G || li >= hdr(o)[0]) {
                check(false, "ring position outside every owner's rows", g);
                continue;
            }
            L[n0 + loc] = tab[(size_t)hdr(o)[kMJHOwn] + li];
            bool near = o == g;
            for (int q = 0; q < hd[kMJHCount]; ++q) near |= hd[kMJHNb + q] == o;
            check(near, "a ring read from a workgroup outside the neighbour set", g);
        }
        for (int h = 0; h < nh; ++h) check(rg[h] == L[n0 + h], "ring row's state differs from its position's", g);
        int32_t cc[W];
        float vv[W], lo;
        for (int i = 0; i < n0; ++i) {
            entries(og[i], cc, vv, lo);
            for (int e = 0; e < W; ++e) {
                const int l = ol[(size_t)i * W + e];
                check(l >= 0 && l < nS[1] && L[l] == cc[e], "own row's local column", g);
            }
        }
        for (int h = 0; h < nh; ++h) {
            entries(rg[h], cc, vv, lo);
            int r = 1;  // ring of this row: it reads rings <= r + 1 only
            while (n0 + h >= nS[r]) ++r;
            for (int e = 0; e < W; ++e) {
                const int l = rl[(size_t)h * W + e];
                check(l >= 0 && l < nS[r + 1] && L[l] == cc[e], "ring row's local column", g);
            }
        }
    }
    if (bad) {
        std::printf("table checks failed: %ld\n", bad);
        return 1;
    }

    // rounds: exchange buffers in tile order, per-workgroup LDS images whose
    // values carry the step they hold
    std::mt19937_64 rng(5);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::vector<double> ref(n), tmp(n);
    for (auto& v : ref) v = U(rng);
    std::vector<double> xa((size_t)G * kMJOwn, -1.0), xb = xa;
    std::vector<std::vector<double>> own(G);
    for (int g = 0; g < G; ++g) {
        const int n0 = hdr(g)[0];
        own[g].resize(n0);
        const int32_t* og = tab.data() + hdr(g)[kMJHOwn];
        for (int i = 0; i < n0; ++i) own[g][i] = xa[(size_t)g * kMJOwn + i] = ref[og[i]];
    }
    auto jump_all = [&](const std::vector<double>& a, std::vector<double>& b) {
        int32_t cc[W];
        float vv[W], lo;
        for (int64_t m = 0; m < n; ++m) {
            entries(m, cc, vv, lo);
            double acc = (double)lo * a[m];
            acc = std::fma((double)vv[0], a[m], acc);
            for (int e = 1; e < W; ++e) acc = std::fma((double)vv[e], a[cc[e]], acc);
            b[m] = acc;
        }
    };
    long stale = 0;
    for (int q = 0; q < rounds; ++q) {
        const int k = q * S;
        for (int g = 0; g < G; ++g) {
            const int32_t* hd = hdr(g);
            int nS[9];
            for (int j = 0; j <= S; ++j) nS[j] = hd[j];
            const int n0 = nS[0], nh = nS[S - 1] - n0, nl = nS[S] - n0;
            const int32_t* og = tab.data() + hd[kMJHOwn];
            const int32_t* ol = og + n0;
            const int32_t* rg = tab.data() + hd[kMJHRing];
            const int32_t* rl = rg + nh;
            const int32_t* ps = tab.data() + hd[kMJHPos];
            std::vector<double> X[2] = {std::vector<double>(kX, 0.0), std::vector<double>(kX, 0.0)};
            std::vector<int> T[2] = {std::vector<int>(kX, -1), std::vector<int>(kX, -1)};
            for (int i = 0; i < n0; ++i) {
                X[0][i] = own[g][i];
                T[0][i] = k;
            }
            for (int h = 0; h < nl; ++h) {
                X[0][n0 + ps[nl + h]] = xa[ps[h]];
                T[0][n0 + ps[nl + h]] = k;
            }
            auto rd = [&](int buf, int l, int want) {
                if (T[buf][l] != want) ++stale;
                return X[buf][l];
            };
            int32_t cc[W];
            float vv[W], lo;
            for (int jj = 1; jj <= S; ++jj) {
                const int rb = (jj & 1) ? 0 : 1, wb = rb ^ 1;
                std::vector<std::pair<int, double>> out;
                for (int i = 0; i < n0; ++i) {
                    entries(og[i], cc, vv, lo);
                    const double self = rd(rb, i, k + jj - 1);
                    double acc = (double)lo * self;
                    acc = std::fma((double)vv[0], self, acc);
                    for (int e = 1; e < W; ++e) acc = std::fma((double)vv[e], rd(rb, ol[(size_t)i * W + e], k + jj - 1), acc);
                    out.emplace_back(i, acc);
                }
                for (int h = 0; h < nS[S - jj] - n0; ++h) {
                    entries(rg[h], cc, vv, lo);
                    double acc = (double)lo * rd(rb, rl[(size_t)h * W], k + jj - 1);
                    for (int e = 0; e < W; ++e) acc = std::fma((double)vv[e], rd(rb, rl[(size_t)h * W + e], k + jj - 1), acc);
                    out.emplace_back(n0 + h, acc);
                }
                for (const auto& o : out) {
                    X[wb][o.first] = o.second;
                    T[wb][o.first] = k + jj;
                }
            }
            for (int i = 0; i < n0; ++i) {
                if (T[0][i] != k + S) ++stale;
                own[g][i] = xb[(size_t)g * kMJOwn + i] = X[0][i];
            }
        }
        std::swap(xa, xb);
        for (int j = 0; j < S; ++j) {
            jump_all(ref, tmp);
            std::swap(ref, tmp);
        }
    }
    double maxd = 0.0;
    for (int64_t m = 0; m < n; ++m) maxd = std::max(maxd, std::fabs(own[owner[m]][place[m]] - ref[m]));
    std::printf("G=%d rounds=%d stale reads=%ld max |tiled - whole| = %.3g\n", G, rounds, stale, maxd);
    return stale == 0 && maxd == 0.0 ? 0 : 1;
}
