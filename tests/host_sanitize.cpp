// Host-side checks of the library's host-only entry points, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code (see
// test_host_sanitizer.py): grid validation, rectilinear axis tables, the well
// and indicator partition builders, face-list conversion, footprint estimates
// and the early error paths of set-up, on seeded random grids and on malformed inputs.  Every
// call must return a status (never crash, read out of bounds or overflow);
// valid inputs must be accepted and malformed ones rejected.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "msrsb.h"

namespace {

uint64_t g_state = 0x2001016240000001ULL;
uint32_t rnd() {  // 64-bit LCG (Knuth's MMIX constants), upper bits
    g_state = g_state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (uint32_t)(g_state >> 33);
}
int rint_(int lo, int hi) { return lo + (int)(rnd() % (uint32_t)(hi - lo + 1)); }
double runit() { return (rnd() + 0.5) / 2147483648.0; }

int g_fail = 0;
void expect(bool ok, const char *what, int line) {
    if (!ok) {
        std::fprintf(stderr, "FAILED line %d: %s (last error: %s)\n", line, what, msrsb_last_error());
        ++g_fail;
    }
}
#define EXPECT(c) expect((c), #c, __LINE__)

struct Box {
    int nx, ny, nz;
    std::vector<uint8_t> active, fault;
    std::vector<double> tx, ty, tz, src, bct, bcv;
    std::vector<int32_t> bcc;
    msrsb_grid g{};
    int N() const { return nx * ny * nz; }
    void wire() {
        g.nx = nx; g.ny = ny; g.nz = nz;
        g.active = active.data();
        g.tx = tx.data(); g.ty = ty.data(); g.tz = tz.data();
        g.fault = fault.data();
        g.n_bc = (int32_t)bcc.size();
        g.bc_cell = bcc.data(); g.bc_trans = bct.data(); g.bc_value = bcv.data();
        g.source = src.data();
    }
};

// A random box: active mask (at least one active cell), face T zero on the
// box boundary and at inactive cells, random fault flags, sources, and a
// Dirichlet connection on every connected piece.
Box random_box(int maxd) {
    Box b;
    b.nx = rint_(1, maxd); b.ny = rint_(1, maxd); b.nz = rint_(1, maxd);
    const int N = b.N(), nx = b.nx, ny = b.ny, nz = b.nz;
    b.active.assign(N, 1);
    for (int i = 0; i < N; ++i)
        if (rnd() % 10 == 0) b.active[i] = 0;
    bool any = false;
    for (int i = 0; i < N; ++i) any = any || b.active[i];
    if (!any) b.active[0] = 1;
    b.tx.assign(N, 0.0); b.ty.assign(N, 0.0); b.tz.assign(N, 0.0);
    for (int i = 0; i < N; ++i) {
        const int x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
        if (!b.active[i]) continue;
        if (x + 1 < nx && b.active[i + 1]) b.tx[i] = runit();
        if (y + 1 < ny && b.active[i + nx]) b.ty[i] = runit();
        if (z + 1 < nz && b.active[i + nx * ny]) b.tz[i] = runit();
    }
    b.fault.assign((size_t)3 * N, 0);
    for (auto &f : b.fault) f = rnd() % 7 == 0;
    b.src.assign(N, 0.0);
    for (int i = 0; i < N; ++i)
        if (b.active[i]) b.src[i] = runit() - 0.5;
    // one Dirichlet connection on the first cell of every connected piece
    // (face-connected active cells), so that the operator is nonsingular
    std::vector<int> comp(N, -1), stack;
    for (int i = 0; i < N; ++i) {
        if (!b.active[i] || comp[i] >= 0) continue;
        comp[i] = i;
        stack.assign(1, i);
        while (!stack.empty()) {
            const int c = stack.back();
            stack.pop_back();
            const int nb[6] = {c + 1, c - 1, c + nx, c - nx, c + nx * ny, c - nx * ny};
            const double t[6] = {b.tx[c], c >= 1 ? b.tx[c - 1] : 0.0, b.ty[c], c >= nx ? b.ty[c - nx] : 0.0,
                                 b.tz[c], c >= nx * ny ? b.tz[c - nx * ny] : 0.0};
            for (int q = 0; q < 6; ++q)
                if (t[q] > 0.0 && comp[nb[q]] < 0) {
                    comp[nb[q]] = i;
                    stack.push_back(nb[q]);
                }
        }
        b.bcc.push_back(i);
        b.bct.push_back(1.0 + runit());
        b.bcv.push_back(runit());
    }
    b.wire();
    return b;
}

void check_axis_support() {
    for (int n = 1; n <= 40; ++n)
        for (int m = 1; m <= n; ++m) {
            std::vector<int32_t> lo(n), nv(n), slo(m), shi(m);
            EXPECT(msrsb_axis_support(n, m, lo.data(), nv.data(), slo.data(), shi.data()) == MSRSB_OK);
            for (int i = 0; i < n; ++i) EXPECT(lo[i] >= 0 && lo[i] < m && (nv[i] == 1 || nv[i] == 2) && lo[i] + nv[i] <= m);
            for (int J = 0; J < m; ++J) EXPECT(slo[J] >= 0 && slo[J] <= shi[J] && shi[J] < n);
            EXPECT(msrsb_axis_support(n, m, nullptr, nullptr, nullptr, nullptr) == MSRSB_OK);
        }
    std::vector<int32_t> t(8);
    EXPECT(msrsb_axis_support(5, 0, t.data(), t.data(), t.data(), t.data()) != MSRSB_OK);
    EXPECT(msrsb_axis_support(5, 6, t.data(), t.data(), t.data(), t.data()) != MSRSB_OK);
    EXPECT(msrsb_axis_support(0, 1, t.data(), t.data(), t.data(), t.data()) != MSRSB_OK);
}

void check_validation() {
    for (int rep = 0; rep < 200; ++rep) {
        Box b = random_box(7);
        EXPECT(msrsb_validate_grid(&b.g) == MSRSB_OK);
        const int N = b.N();
        // malformed copies, one defect each
        {
            Box c = b;
            c.tx[rint_(0, N - 1)] = -1.0;
            c.wire();
            EXPECT(msrsb_validate_grid(&c.g) != MSRSB_OK);
        }
        {
            Box c = b;
            const int y = rint_(0, c.ny - 1), z = rint_(0, c.nz - 1);
            c.tx[(c.nx - 1) + c.nx * (y + c.ny * z)] = 1.0;  // face beyond the box
            c.wire();
            EXPECT(msrsb_validate_grid(&c.g) != MSRSB_OK);
        }
        {
            Box c = b;
            c.tz[rint_(0, N - 1)] = std::nan("");
            c.wire();
            EXPECT(msrsb_validate_grid(&c.g) != MSRSB_OK);
        }
        {
            Box c = b;
            c.bcc[0] = N + rint_(0, 5);
            c.wire();
            EXPECT(msrsb_validate_grid(&c.g) != MSRSB_OK);
        }
        {
            Box c = b;
            c.bcc[0] = -1 - rint_(0, 5);
            c.wire();
            EXPECT(msrsb_validate_grid(&c.g) != MSRSB_OK);
        }
        {
            Box c = b;
            c.bct[0] = -0.5;
            c.wire();
            EXPECT(msrsb_validate_grid(&c.g) != MSRSB_OK);
        }
        {
            Box c = b;
            c.g.n_bc = -3;
            EXPECT(msrsb_validate_grid(&c.g) != MSRSB_OK);
        }
        {
            Box c = b;
            c.g.tx = nullptr;
            EXPECT(msrsb_validate_grid(&c.g) != MSRSB_OK);
        }
        {
            Box c = b;
            c.g.nx = 0;
            EXPECT(msrsb_validate_grid(&c.g) != MSRSB_OK);
        }
    }
    EXPECT(msrsb_validate_grid(nullptr) != MSRSB_OK);
}

void check_wells() {
    for (int rep = 0; rep < 150; ++rep) {
        Box b = random_box(9);
        const int N = b.N();
        std::vector<int> act;
        for (int i = 0; i < N; ++i)
            if (b.active[i]) act.push_back(i);
        const int nw = rint_(1, 4);
        std::vector<int32_t> ptr{0}, cells;
        for (int w = 0; w < nw; ++w) {
            const int k = rint_(1, 3);
            for (int q = 0; q < k; ++q) cells.push_back(act[rint_(0, (int)act.size() - 1)]);
            ptr.push_back((int32_t)cells.size());
        }
        std::vector<int32_t> block(N, -7);
        const int radius = rint_(0, 3);
        EXPECT(msrsb_partition_wells(&b.g, nw, ptr.data(), cells.data(), radius, block.data()) == MSRSB_OK);
        for (int i = 0; i < N; ++i) EXPECT(b.active[i] ? (block[i] >= 0 && block[i] <= nw) : block[i] == -1);
        // malformed: a cell outside the grid, an inactive cell, an empty well, NULL output
        std::vector<int32_t> bad = cells;
        bad[0] = N + 2;
        EXPECT(msrsb_partition_wells(&b.g, nw, ptr.data(), bad.data(), radius, block.data()) != MSRSB_OK);
        for (int i = 0; i < N; ++i)
            if (!b.active[i]) {
                bad = cells;
                bad[0] = i;
                EXPECT(msrsb_partition_wells(&b.g, nw, ptr.data(), bad.data(), radius, block.data()) != MSRSB_OK);
                break;
            }
        std::vector<int32_t> eptr = ptr;
        eptr[1] = eptr[0];
        if (nw == 1) EXPECT(msrsb_partition_wells(&b.g, nw, eptr.data(), cells.data(), radius, block.data()) != MSRSB_OK);
        EXPECT(msrsb_partition_wells(&b.g, nw, ptr.data(), cells.data(), radius, nullptr) != MSRSB_OK);
        EXPECT(msrsb_partition_wells(&b.g, nw, ptr.data(), cells.data(), -1, block.data()) != MSRSB_OK);
    }
}

void check_indicator() {
    for (int rep = 0; rep < 150; ++rep) {
        Box b = random_box(9);
        const int N = b.N();
        std::vector<double> ind(N);
        for (auto &v : ind) v = rnd() % 5 == 0 ? (double)rint_(0, 3) : std::log(runit());  // ties included
        const int32_t cd[3] = {rint_(1, b.nx), rint_(1, b.ny), rint_(1, b.nz)};
        std::vector<int32_t> block(N, -7);
        const int nb = rint_(1, 5), mc = rint_(0, 12);
        EXPECT(msrsb_partition_indicator(&b.g, ind.data(), nb, cd, mc, block.data()) == MSRSB_OK);
        int first_active = -1;
        for (int i = 0; i < N; ++i) {
            EXPECT(b.active[i] ? block[i] >= 0 && block[i] < N : block[i] == -1);
            if (b.active[i] && first_active < 0) first_active = i;
        }
        std::vector<double> bad = ind;
        bad[first_active] = std::nan("");
        EXPECT(msrsb_partition_indicator(&b.g, bad.data(), nb, cd, mc, block.data()) != MSRSB_OK);
        const int32_t cdbad[3] = {b.nx + 1, 1, 1};
        EXPECT(msrsb_partition_indicator(&b.g, ind.data(), nb, cdbad, mc, block.data()) != MSRSB_OK);
        EXPECT(msrsb_partition_indicator(&b.g, ind.data(), 0, cd, mc, block.data()) != MSRSB_OK);
        EXPECT(msrsb_partition_indicator(&b.g, nullptr, nb, cd, mc, block.data()) != MSRSB_OK);
    }
}

void check_faces_to_box() {
    for (int rep = 0; rep < 150; ++rep) {
        Box b = random_box(9);
        const int N = b.N(), nx = b.nx, nxy = b.nx * b.ny;
        std::vector<int32_t> fc;
        std::vector<double> ft;
        const std::vector<double> *T[3] = {&b.tx, &b.ty, &b.tz};
        const int step[3] = {1, nx, nxy};
        for (int a = 0; a < 3; ++a)
            for (int i = 0; i < N; ++i)
                if ((*T[a])[i] != 0.0) {
                    fc.push_back(i);
                    fc.push_back(i + step[a]);
                    ft.push_back((*T[a])[i]);
                }
        const int F = (int)ft.size();
        std::vector<double> tx(N, -1.0), ty(N, -1.0), tz(N, -1.0);
        EXPECT(msrsb_faces_to_box(b.nx, b.ny, b.nz, F, fc.data(), ft.data(), tx.data(), ty.data(), tz.data()) ==
               MSRSB_OK);
        EXPECT(tx == b.tx && ty == b.ty && tz == b.tz);
        if (F > 0) {  // one defect each
            const int f = rint_(0, F - 1);
            std::vector<int32_t> bad = fc;
            bad[2 * f + 1] = N + rint_(0, 3);
            EXPECT(msrsb_faces_to_box(b.nx, b.ny, b.nz, F, bad.data(), ft.data(), tx.data(), ty.data(), tz.data()) !=
                   MSRSB_OK);
            bad = fc;
            std::swap(bad[2 * f], bad[2 * f + 1]);
            EXPECT(msrsb_faces_to_box(b.nx, b.ny, b.nz, F, bad.data(), ft.data(), tx.data(), ty.data(), tz.data()) !=
                   MSRSB_OK);
            std::vector<double> badt = ft;
            badt[f] = -1.0;
            EXPECT(msrsb_faces_to_box(b.nx, b.ny, b.nz, F, fc.data(), badt.data(), tx.data(), ty.data(), tz.data()) !=
                   MSRSB_OK);
            std::vector<int32_t> dup = fc;
            dup.push_back(fc[2 * f]);
            dup.push_back(fc[2 * f + 1]);
            std::vector<double> dupt = ft;
            dupt.push_back(1.0);
            EXPECT(msrsb_faces_to_box(b.nx, b.ny, b.nz, F + 1, dup.data(), dupt.data(), tx.data(), ty.data(),
                                      tz.data()) != MSRSB_OK);
        }
        EXPECT(msrsb_faces_to_box(b.nx, b.ny, b.nz, 1, nullptr, ft.data(), tx.data(), ty.data(), tz.data()) !=
               MSRSB_OK);
        EXPECT(msrsb_faces_to_box(0, b.ny, b.nz, 0, fc.data(), ft.data(), tx.data(), ty.data(), tz.data()) !=
               MSRSB_OK);
    }
}

void check_footprint_and_setup_errors() {
    for (int rep = 0; rep < 100; ++rep) {
        Box b = random_box(8);
        const int N = b.N();
        msrsb_options o;
        msrsb_default_options(&o);
        o.smoother = rint_(0, 2);
        o.precision = rint_(0, 1);
        o.outer = rint_(0, 1);
        o.restart = rint_(1, 64);
        std::vector<int32_t> ids(N);
        for (auto &v : ids) v = rint_(0, 9);
        msrsb_partition p[3] = {};
        p[0].kind = MSRSB_PART_CARTESIAN;
        p[0].coarse_dims[0] = rint_(1, b.nx); p[0].coarse_dims[1] = rint_(1, b.ny); p[0].coarse_dims[2] = rint_(1, b.nz);
        p[1].kind = MSRSB_PART_GRAPH;
        p[1].block_of_cell = ids.data();
        p[1].overlap = rint_(0, 3);
        p[2].kind = MSRSB_PART_FAULT_CUT;
        p[2].parent = 0;
        const size_t fb = msrsb_footprint_bytes(&b.g, 3, p, &o);
        EXPECT(fb > (size_t)N * 8);
        // set-up errors that are found before any device work
        msrsb_ctx *ctx = nullptr;
        EXPECT(msrsb_setup(&b.g, 3, p, &o, nullptr, nullptr, nullptr) != MSRSB_OK);
        msrsb_options ob = o;
        ob.omega = 3.0;
        EXPECT(msrsb_setup(&b.g, 3, p, &ob, nullptr, nullptr, &ctx) != MSRSB_OK && ctx == nullptr);
        ob = o;
        ob.smoother = 9;
        EXPECT(msrsb_setup(&b.g, 3, p, &ob, nullptr, nullptr, &ctx) != MSRSB_OK && ctx == nullptr);
        msrsb_partition q[3] = {p[0], p[1], p[2]};
        q[0].coarse_dims[0] = b.nx + 1;
        EXPECT(msrsb_setup(&b.g, 3, q, &o, nullptr, nullptr, &ctx) != MSRSB_OK && ctx == nullptr);
        q[0] = p[0];
        q[2].parent = 5;
        EXPECT(msrsb_setup(&b.g, 3, q, &o, nullptr, nullptr, &ctx) != MSRSB_OK && ctx == nullptr);
        q[2] = p[2];
        q[0].kind = 17;
        EXPECT(msrsb_setup(&b.g, 3, q, &o, nullptr, nullptr, &ctx) != MSRSB_OK && ctx == nullptr);
        EXPECT(msrsb_setup(&b.g, 0, p, &o, nullptr, nullptr, &ctx) != MSRSB_OK && ctx == nullptr);
        Box c = b;
        c.tx[0] = -2.0;
        c.wire();
        EXPECT(msrsb_setup(&c.g, 3, p, &o, nullptr, nullptr, &ctx) != MSRSB_OK && ctx == nullptr);
        msrsb_allocator half{};
        EXPECT(msrsb_setup(&b.g, 3, p, &o, &half, nullptr, &ctx) != MSRSB_OK && ctx == nullptr);
        EXPECT(msrsb_last_error() != nullptr);
    }
}

}  // namespace

int main() {
    check_axis_support();
    check_validation();
    check_wells();
    check_indicator();
    check_faces_to_box();
    check_footprint_and_setup_errors();
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("host sanitize ok\n");
    return 0;
}
