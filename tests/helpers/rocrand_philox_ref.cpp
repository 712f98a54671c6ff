// Prints Philox4x32-10 output blocks from rocRAND's engine (host path of its
// public header) for the counters/keys read from stdin, one block per line:
//   input : key_lo key_hi subsequence_lo subsequence_hi block_index   (hex)
//   output: x0 x1 x2 x3                                              (hex)
// rocRAND's engine holds the counter as (block_lo, block_hi, subseq_lo,
// subseq_hi) and the key as (seed_lo, seed_hi).  Used only by the test suite.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned klo, khi, slo, shi, blk;
    while (std::scanf("%x %x %x %x %x", &klo, &khi, &slo, &shi, &blk) == 5) {
        unsigned long long seed = ((unsigned long long)khi << 32) | klo;
        unsigned long long subseq = ((unsigned long long)shi << 32) | slo;
        rocrand_device::philox4x32_10_engine eng(seed, subseq, 4ull * blk);
        uint4 r = eng.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
