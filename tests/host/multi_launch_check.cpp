// Host-only checks of the multi-block launch tables of the batched path
// (paper_2105_13678_amd/csrc/pa_multi.hpp): for random sets of blocks with
// random grids and argument structs of the sizes the kernels use (including
// sizes that are not multiples of 16), every workgroup of the launch is
// located (with the lookup the kernels run) at exactly one position of
// exactly one block's grid, padding workgroups only fill the gaps before
// 8-aligned starts, and the argument struct found at sizeof(Args) stride is
// that block's.  Built and run by tests/test_host_checks.py; prints "ok".
#include <cstdio>
#include <cstdlib>
#include <set>
#include <tuple>
#include <vector>

#include "pa_multi.hpp"

static int failures = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c) && failures++ < 20) std::printf("FAILED line %d: %s\n", __LINE__, #c); \
    } while (0)

int main() {
    std::srand(2105);
    const size_t sizes[] = {8, 24, 88, 232, 344, 360, 408, 504};
    for (int trial = 0; trial < 300; ++trial) {
        const size_t args_size = sizes[std::rand() % 8];
        const size_t nm = 1 + std::rand() % 70;
        std::vector<std::vector<unsigned char>> bytes(nm);
        std::vector<pa::MultiMember> mem(nm);
        for (size_t m = 0; m < nm; ++m) {
            bytes[m].resize(args_size);
            for (size_t b = 0; b < args_size; ++b) bytes[m][b] = (unsigned char)(m * 131 + b * 7 + trial);
            const uint32_t gx = 1 + std::rand() % (trial % 3 ? 40 : 2000), gy = 1 + std::rand() % 5,
                           gz = 1 + std::rand() % 3;
            mem[m] = pa::MultiMember{gx, gy, gz, bytes[m].data()};
        }
        const size_t off0 = std::rand() % 100;
        const pa::MultiLayout L = pa::multi_layout(mem, args_size, off0);
        CHECK(L.o_args % 16 == 0 && L.o_args >= off0 && L.o_geo % 16 == 0 && L.o_owner % 16 == 0);
        CHECK(L.o_geo >= L.o_args + nm * args_size && L.o_owner >= L.o_geo + nm * sizeof(pa::MultiGeo));
        CHECK(L.end >= L.o_owner + (L.total / 8) * 2 && L.total % 8 == 0);
        std::vector<unsigned char> buf(L.end + 64, 0xEE);
        pa::multi_fill(mem, args_size, L, buf.data());
        const pa::MultiGeo *geo = (const pa::MultiGeo *)(buf.data() + L.o_geo);
        const uint16_t *owner = (const uint16_t *)(buf.data() + L.o_owner);
        std::set<std::tuple<uint32_t, uint32_t, uint32_t, uint32_t>> seen;
        size_t real = 0;
        for (uint32_t w = 0; w < L.total; ++w) {
            uint32_t x = 0, y = 0, z = 0;
            const uint32_t i = pa::multi_locate(geo, owner, w, &x, &y, &z);
            if (i == pa::MULTI_NONE) continue;
            CHECK(i < nm);
            if (i >= nm) break;
            CHECK(x < mem[i].gx && y < mem[i].gy && z < mem[i].gz);
            CHECK(seen.insert(std::make_tuple(i, x, y, z)).second);
            CHECK(geo[i].start % 8 == 0 && w >= geo[i].start);
            ++real;
        }
        size_t want = 0;
        for (const auto &m : mem) want += (size_t)m.gx * m.gy * m.gz;
        CHECK(real == want && seen.size() == want);
        // padding only in the gaps: at most 7 workgroups per block
        CHECK(L.total - want <= 8 * nm);
        // the argument struct of block i at the kernels' stride sizeof(Args)
        for (size_t m = 0; m < nm; ++m)
            CHECK(std::equal(bytes[m].begin(), bytes[m].end(), buf.begin() + L.o_args + m * args_size));
    }
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
