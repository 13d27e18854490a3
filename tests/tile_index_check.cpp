// Host-side bounds check of the LDS and workspace indices the tile march and
// the staged streaming kernels form, for every tile edge, using the same
// index helpers the kernels use (fmm_tile.h).  Prints one line per failure
// and exits non-zero if there is any; "ok" otherwise.
#include <cstdio>
#include <set>

#include "fmm_tile.h"

using namespace fmm;

static int failures = 0;
#define CHECK(cond, ...)                                                     \
    do {                                                                     \
        if (!(cond)) {                                                       \
            if (failures < 20) std::printf("FAIL E=%d: %s\n", E, #cond);  \
            failures++;                                                      \
        }                                                                    \
    } while (0)

// Block coordinates (each in [-1, E]) of block index d.
template <int E> static void coords(int d, int c[3])
{
    using Gm = Geo<E>;
    c[2] = d % Gm::D - 1;
    c[1] = (d / Gm::D) % Gm::D - 1;
    c[0] = d / (Gm::D * Gm::D) - 1;
}

template <int E> static int n_out(const int c[3])
{
    int n = 0;
    for (int a = 0; a < 3; a++) n += (c[a] < 0 || c[a] >= E);
    return n;
}

template <int E> static void check_tile()
{
    using Gm = Geo<E>;
    constexpr int V = Gm::V, DV = Gm::DV, FACE = Gm::FACE;
    const int off[6] = {-Gm::OX, Gm::OX, -Gm::OY, Gm::OY, -Gm::OZ, Gm::OZ};
    // the halo cells a tile load writes: every face cell exactly once
    std::set<int> halo;
    for (int q = 0; q < 6 * FACE; q++) {
        const int f = q / FACE, uv = q - f * FACE, u = uv / E, w = uv - u * E;
        int c0, c1, c2;
        face_cell<E>(f, u, w, c0, c1, c2);
        const int d = Gm::dom(c0, c1, c2);
        CHECK(d >= 0 && d < DV);
        int c[3];
        coords<E>(d, c);
        CHECK(n_out<E>(c) == 1);
        CHECK(halo.insert(d).second);
        // the interior cell next to it, and its interior index
        face_inner<E>(f, c0, c1, c2);
        CHECK(c0 >= 0 && c0 < E && c1 >= 0 && c1 < E && c2 >= 0 && c2 < E);
        const int pi = (c0 * E + c1) * E + c2;
        CHECK(pi >= 0 && pi < V);
        const int di = Gm::dom(c0, c1, c2);
        CHECK(di - d == -off[f] || di - d == off[f]);
        CHECK(Gm::domp(pi) == di);
        // the cell of the neighbouring tile this halo cell copies
        const int ax = f >> 1;
        const bool plus = f & 1;
        int cc[3];
        face_cell<E>(f, u, w, cc[0], cc[1], cc[2]);
        const int n0c = ax == 0 ? (plus ? 0 : E - 1) : cc[0];
        const int n1c = ax == 1 ? (plus ? 0 : E - 1) : cc[1];
        const int n2c = ax == 2 ? (plus ? 0 : E - 1) : cc[2];
        CHECK(n0c >= 0 && n0c < E && n1c >= 0 && n1c < E && n2c >= 0 && n2c < E);
        CHECK((n0c * E + n1c) * E + n2c < V);
        if (ax == 2) CHECK(n0c * E + n1c < FACE);
    }
    CHECK((int)halo.size() == 6 * FACE);
    for (int p = 0; p < V; p++) {
        const int d = Gm::domp(p);
        CHECK(d >= 0 && d < DV);
        int c[3];
        coords<E>(d, c);
        CHECK(n_out<E>(c) == 0);
        CHECK((c[0] * E + c[1]) * E + c[2] == p);
        const int i0 = p >> (2 * Gm::LOG), i1 = (p >> Gm::LOG) & (E - 1), i2 = p & (E - 1);
        CHECK(i0 == c[0] && i1 == c[1] && i2 == c[2]);
        const int step[6] = {-E * E, E * E, -E, E, -1, 1};
        const bool guard[6] = {i0 > 0, i0 < E - 1, i1 > 0, i1 < E - 1, i2 > 0, i2 < E - 1};
        for (int k = 0; k < 6; k++) {
            // every stencil read of an interior cell is an interior cell or a
            // loaded face-halo cell (never an edge or corner of the block)
            const int nd = d + off[k];
            CHECK(nd >= 0 && nd < DV);
            int cn[3];
            coords<E>(nd, cn);
            CHECK(n_out<E>(cn) <= 1);
            if (n_out<E>(cn) == 1) CHECK(halo.count(nd) == 1);
            // the relaxation marks interior index p + step only under its
            // coordinate guard, and then it is that neighbour; without the
            // guard the neighbour is a halo cell (mark_nbrs relies on halo
            // cells never carrying the updatable flag there)
            if (guard[k]) {
                const int q = p + step[k];
                CHECK(q >= 0 && q < V);
                CHECK(Gm::domp(q) == nd);
            } else {
                CHECK(n_out<E>(cn) == 1);
            }
        }
        // write-back of the axis-2 faces
        if (i2 == 0 || i2 == E - 1) CHECK(i0 * E + i1 < FACE);
    }
    // the spare dwords of the candidate bytes: one per lane, past the
    // interior flags (which alone the compaction reads), in distinct banks
    {
        std::set<int> banks;
        for (int lane = 0; lane < 64; lane++) {
            const int s = Gm::spare(lane);
            CHECK(s >= V && s + 3 < Gm::CFB && s % 4 == 0);
            if (lane < 32) CHECK(banks.insert((s / 4) % 32).second);
        }
    }
    // byte-flag compaction of a one-wavefront group: 64 lanes of K flags
    if (Gm::K % 8 == 0) {
        CHECK(64 * Gm::K == V);
        for (int lane = 0; lane < 64; lane++)
            for (int j = 0; j < Gm::K / 8; j++)
                for (int bit = 0; bit < 8; bit++) CHECK(lane * Gm::K + j * 8 + bit < V);
    } else {
        for (int lane = 0; lane < 64; lane++)
            if (lane * Gm::K < V)
                for (int j = 0; j < Gm::K; j++) CHECK(lane * Gm::K + j < V + 64);
    }
}

// Bit-flag compaction of a workgroup group of G threads: thread r owns C =
// V / G cells starting at r C, i.e. bits (r C) % 32 .. of word (r C) / 32;
// its wavefront w writes its candidates to list entries [w 64 C, (w + 1) 64 C).
template <int E, int G> static void check_bits()
{
    constexpr int V = Geo<E>::V, C = V / G;
    CHECK(V % G == 0 && C >= 1 && C <= 32 && 32 % C == 0);
    for (int r = 0; r < G; r++) {
        const int word = (r * C) >> 5, sh = (r * C) & 31;
        CHECK(word >= 0 && word < V / 32);
        CHECK(sh + C <= 32);
        // the threads sharing a word are in one wavefront
        CHECK(((word * 32) / C) / 64 == r / 64);
        const int w = r / 64;
        CHECK(w * 64 * C + 64 * C <= V);
    }
}

template <int E, typename T> static void check_stage()
{
    using S = Stage<E, T>;
    CHECK((S::R * S::W) % STAGE_THREADS == 0 && (S::CH * S::V) % STAGE_THREADS == 0);
    for (int idx = 0; idx < S::R * S::W; idx++) {
        const int r = idx / S::W, c = idx - r * S::W, k = c / E;
        const int li = k * S::TS + r * E + c % E;
        CHECK(k < S::CH && li >= 0 && li < S::CH * S::TS && r * E + c % E < S::V);
    }
    for (int idx = 0; idx < S::CH * S::V; idx++) {
        const int k = idx / S::V;
        CHECK(k * S::TS + (idx - k * S::V) < S::CH * S::TS);
    }
    CHECK(S::CH * S::TS * (int)sizeof(T) <= 160 * 1024);
}

#undef CHECK

int main()
{
    check_tile<4>();
    check_tile<8>();
    check_tile<16>();
    check_bits<16, 256>();
    check_bits<16, 512>();
    check_stage<4, float>();
    check_stage<4, double>();
    check_stage<8, float>();
    check_stage<8, double>();
    check_stage<16, float>();
    check_stage<16, double>();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
