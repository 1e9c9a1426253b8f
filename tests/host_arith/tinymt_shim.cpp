// Host build of the library's TinyMT32 arithmetic (tinymt_arith.hpp) for CPU
// tests: the generator, the parameter checks, the jump tables and the stream
// placement, each compared with the oracle without a GPU.
#include <stdint.h>
#include "tinymt_arith.hpp"

using namespace mrg::tmt;

extern "C" {

// n tempered outputs of a state under parameters p; s is advanced.
void tshim_draw(uint32_t *s, const uint32_t *p, uint64_t n, uint32_t *out)
{
    for (uint64_t k = 0; k < n; ++k) {
        step(s, p[0], p[1]);
        out[k] = temper(s[0], s[2], s[3], p[2]);
    }
}

void tshim_seed(uint32_t seed, const uint32_t *p, uint32_t *s) { seed_status(seed, p[0], p[1], p[2], s); }

void tshim_candidate(uint64_t master, uint64_t c, uint32_t *p) { candidate(master, c, p); }

int tshim_charpoly(const uint32_t *p, uint32_t *phi) { return charpoly(p, phi); }

int tshim_irreducible(const uint32_t *phi) { return irreducible127(phi) ? 1 : 0; }

int tshim_params_ok(const uint32_t *p)
{
    uint32_t phi[4];
    return params_ok(p, phi) ? 1 : 0;
}

void tshim_mulmod(const uint32_t *a, const uint32_t *b, const uint32_t *phi, uint32_t *r)
{
    mulmod(a, b, phi, r);
}

void tshim_pow_table(const uint32_t *phi, uint32_t *pow) { pow_table(phi, pow); }

// s <- T^e s (e as three little-endian words)
void tshim_jump(uint32_t *s, const uint32_t *p, const uint32_t *phi, const uint32_t *pow,
                const uint64_t *e)
{
    jump(s, p[0], p[1], phi, pow, e[0], e[1], e[2]);
}

float tshim_to_f32(uint32_t w) { return to_f32(w); }
double tshim_to_f64(uint32_t w) { return to_f64(w); }

}  // extern "C"
