// Independent reference for the oracle's Philox4x32-10: runs rocRAND's host-callable
// philox4x32_10 engine (header-only, compiled here from its installed source) on given
// (counter, key) pairs.  With seed = key, subsequence = c2 + 2^32 c3 and
// offset = 4 (c0 + 2^32 c1) the engine's next four outputs are Philox(counter, key).
// Usage: rocrand_philox_ref <in.bin> <out.bin>; in = count x (c0,c1,c2,c3,k0,k1) uint32.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>
#include <cstdio>
#include <vector>

int main(int argc, char** argv)
{
    if (argc != 3) return 2;
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 3;
    std::vector<uint32_t> in;
    uint32_t buf[6];
    while (std::fread(buf, sizeof(uint32_t), 6, f) == 6) in.insert(in.end(), buf, buf + 6);
    std::fclose(f);
    size_t count = in.size() / 6;
    std::vector<uint32_t> out(4 * count);
    for (size_t i = 0; i < count; ++i) {
        const uint32_t* r = &in[6 * i];
        unsigned long long seed = (unsigned long long)r[4] | ((unsigned long long)r[5] << 32);
        unsigned long long sub = (unsigned long long)r[2] | ((unsigned long long)r[3] << 32);
        unsigned long long off = 4ull * ((unsigned long long)r[0] | ((unsigned long long)r[1] << 32));
        rocrand_device::philox4x32_10_engine eng(seed, sub, off);
        for (int k = 0; k < 4; ++k) out[4 * i + k] = eng.next();
    }
    FILE* g = std::fopen(argv[2], "wb");
    if (!g) return 4;
    std::fwrite(out.data(), sizeof(uint32_t), out.size(), g);
    std::fclose(g);
    return 0;
}
