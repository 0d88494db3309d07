// Host-only driver of the stencil builder and the packing routines of
// libmlbm.so, for sanitizer builds (AddressSanitizer, UndefinedBehavior-
// Sanitizer): reads one node set from a binary file, runs every host entry
// point on it and prints checksums of the outputs, which the test compares
// with the same calls on the library built normally.
//
// Input (little-endian): int64 n, int64 n_disks, int32 K, int32 per_departure,
// int32 simple_bounce_back, int32 periodic[2], int32 wall_lo_y, int32 wall_hi_y,
// int32 pad, double lo[2], hi[2], dx, lattice_h, fluid_area, then xy [n][2]
// double, kind [n] uint8, disks [n_disks][3] double.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mlbm.h"

namespace {

template <class T>
bool read(FILE *f, T *dst, size_t count) {
    return std::fread(dst, sizeof(T), count, f) == count;
}

double checksum(const double *v, size_t n) {
    double s = 0;
    for (size_t i = 0; i < n; ++i) s += v[i] * (double)((i % 97) + 1);
    return s;
}

template <class T>
unsigned long long isum(const T *v, size_t n) {
    unsigned long long s = 0;
    for (size_t i = 0; i < n; ++i) s = s * 1000003ull + (unsigned long long)v[i];
    return s;
}

int die(const char *what, int rc) {
    std::fprintf(stderr, "%s failed (%d): %s\n", what, rc, mlbm_last_error());
    return 2;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: %s input.bin\n", argv[0]);
        return 2;
    }
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n = 0, n_disks = 0;
    int32_t ints[8];
    double dbl[7];
    if (!read(f, &n, 1) || !read(f, &n_disks, 1) || !read(f, ints, 8) || !read(f, dbl, 7)) return 2;
    const int32_t K = ints[0], per_departure = ints[1], simple_bb = ints[2];
    std::vector<double> xy(2 * n), disks(3 * n_disks);
    std::vector<uint8_t> kind(n);
    if (!read(f, xy.data(), xy.size()) || !read(f, kind.data(), kind.size()) || !read(f, disks.data(), disks.size()))
        return 2;
    std::fclose(f);

    mlbm_geometry g;
    std::memset(&g, 0, sizeof(g));
    g.n = n;
    g.xy = xy.data();
    g.kind = kind.data();
    g.lo[0] = dbl[0];
    g.lo[1] = dbl[1];
    g.hi[0] = dbl[2];
    g.hi[1] = dbl[3];
    g.periodic[0] = ints[3];
    g.periodic[1] = ints[4];
    g.wall_lo_y = ints[5];
    g.wall_hi_y = ints[6];
    g.n_disks = n_disks;
    g.disks = n_disks ? disks.data() : nullptr;
    g.fluid_area = dbl[6];
    mlbm_stencil_params p;
    std::memset(&p, 0, sizeof(p));
    p.K = K;
    p.reorder = 1;
    p.dx = dbl[4];
    p.n_threads = 4;
    p.lattice_h = dbl[5];
    p.per_departure = per_departure;
    p.simple_bounce_back = simple_bb;

    const size_t rows = per_departure ? 8 * (size_t)K : (size_t)K;
    std::vector<int64_t> perm(n);
    std::vector<int32_t> idx(n * rows);
    std::vector<double> w(n * 8 * (size_t)K), area(n), wl(72);
    std::vector<uint8_t> bb(n), lag(n);
    mlbm_stencils out;
    out.perm = perm.data();
    out.idx = idx.data();
    out.w = w.data();
    out.bb = bb.data();
    out.area = area.data();
    out.lagrange = lag.data();
    out.w_lagrange = wl.data();
    out.n_lagrange = 0;
    int rc = mlbm_build_stencils(&g, &p, &out);
    if (rc) return die("mlbm_build_stencils", rc);
    std::printf("build w %.17g area %.17g wl %.17g idx %llu perm %llu bb %llu lag %llu nlag %lld\n",
                checksum(w.data(), w.size()), checksum(area.data(), area.size()), checksum(wl.data(), wl.size()),
                isum(idx.data(), idx.size()), isum(perm.data(), perm.size()), isum(bb.data(), bb.size()),
                isum(lag.data(), lag.size()), (long long)out.n_lagrange);

    // per-node stencils only: packing, FP16 weights, block marks, tiles
    if (!per_departure) {
        std::vector<uint8_t> kind_new(n);
        for (int64_t i = 0; i < n; ++i) kind_new[i] = kind[perm[i]];
        for (int storage : {MLBM_F64, MLBM_F32}) {
            mlbm_sizes sz;
            rc = mlbm_packed_sizes(n, K, MLBM_POPULATIONS, storage, &sz);
            if (rc) return die("mlbm_packed_sizes", rc);
            std::vector<uint8_t> ip(sz.idx_bytes), wp(sz.w_bytes);
            std::vector<uint16_t> fl(n);
            rc = mlbm_pack_stencils(n, K, storage, idx.data(), w.data(), bb.data(), kind_new.data(), ip.data(),
                                    wp.data(), fl.data());
            if (rc) return die("mlbm_pack_stencils", rc);
            rc = mlbm_mark_lagrange(n, lag.data(), fl.data());
            if (rc) return die("mlbm_mark_lagrange", rc);
            std::printf("pack%d idx %llu w %llu flags %llu\n", storage, isum(ip.data(), ip.size()),
                        isum(wp.data(), wp.size()), isum(fl.data(), fl.size()));
            if (storage == MLBM_F32) {
                std::vector<uint16_t> w16(8 * (size_t)sz.k_padded * n);
                rc = mlbm_weights_to_f16(n, sz.k_padded, (const float *)wp.data(), w16.data());
                if (rc) return die("mlbm_weights_to_f16", rc);
                std::printf("w16 %llu\n", isum(w16.data(), w16.size()));
            }
        }
        for (int tile : {64, 256}) {
            int64_t total = 0;
            int32_t mx = 0;
            rc = mlbm_tile_sizes(n, K, tile, idx.data(), &total, &mx);
            if (rc) return die("mlbm_tile_sizes", rc);
            const int64_t nt = (n + tile - 1) / tile;
            const int64_t k8 = (K + 7) / 8 * 8;
            std::vector<int32_t> hoff(nt + 1), halo(total > 0 ? total : 1);
            std::vector<uint16_t> lidx(k8 * n);
            rc = mlbm_pack_tiles(n, K, tile, idx.data(), hoff.data(), halo.data(), lidx.data());
            if (rc) return die("mlbm_pack_tiles", rc);
            std::printf("tiles%d total %lld max %d halo %llu lidx %llu\n", tile, (long long)total, mx,
                        isum(halo.data(), halo.size()), isum(lidx.data(), lidx.size()));
        }
    }
    return 0;
}
