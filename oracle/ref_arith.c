/*
 * Plain reference arithmetic for the CPU oracle.  TEST INFRASTRUCTURE ONLY:
 * nothing in the product library links or calls this file.
 *
 * Everything here is deliberately textbook: products reduced with the
 * compiler's 128-bit '%', a cyclic radix-2 NTT (bit-reversal permutation
 * followed by butterflies, root powers recomputed by repeated
 * multiplication), and the negacyclic transform obtained the schoolbook way,
 * by twisting the input with powers of psi (a primitive 2n-th root of unity)
 * before the cyclic transform with omega = psi^2.  The negacyclic transform
 * of a is then A_j = sum_i a_i psi^(i(2j+1)) in natural order j.
 *
 * OpenMP is used only across independent polynomials.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

uint64_t oracle_mulmod(uint64_t a, uint64_t b, uint64_t q)
{
    return (uint64_t)(((u128)a * b) % q);
}

uint64_t oracle_powmod(uint64_t b, uint64_t e, uint64_t q)
{
    uint64_t r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = oracle_mulmod(r, b, q);
        b = oracle_mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}

static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q)
{
    return (uint64_t)(((u128)a + b) % q);
}

static uint64_t submod(uint64_t a, uint64_t b, uint64_t q)
{
    return (uint64_t)(((u128)a + q - b) % q);
}

/* In-place cyclic NTT of length n (power of two): A_j = sum_i a_i omega^(ij). */
static void cyclic_ntt(uint64_t *a, size_t n, uint64_t q, uint64_t omega)
{
    for (size_t i = 1, j = 0; i < n; i++) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { uint64_t tmp = a[i]; a[i] = a[j]; a[j] = tmp; }
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        uint64_t wlen = oracle_powmod(omega, n / len, q);
        for (size_t i = 0; i < n; i += len) {
            uint64_t w = 1 % q;
            for (size_t j = 0; j < len / 2; j++) {
                uint64_t u = a[i + j];
                uint64_t v = oracle_mulmod(a[i + j + len / 2], w, q);
                a[i + j] = addmod(u, v, q);
                a[i + j + len / 2] = submod(u, v, q);
                w = oracle_mulmod(w, wlen, q);
            }
        }
    }
}

/* Negacyclic forward transform, natural order: A_j = sum_i a_i psi^(i(2j+1)). */
void oracle_ntt_negacyclic(uint64_t *a, size_t n, uint64_t q, uint64_t psi)
{
    uint64_t p = 1 % q;
    for (size_t i = 0; i < n; i++) {
        a[i] = oracle_mulmod(a[i] % q, p, q);
        p = oracle_mulmod(p, psi, q);
    }
    cyclic_ntt(a, n, q, oracle_mulmod(psi, psi, q));
}

/* Inverse of oracle_ntt_negacyclic. */
void oracle_intt_negacyclic(uint64_t *a, size_t n, uint64_t q, uint64_t psi)
{
    uint64_t psi_inv = oracle_powmod(psi, q - 2, q);
    uint64_t omega_inv = oracle_mulmod(psi_inv, psi_inv, q);
    cyclic_ntt(a, n, q, omega_inv);
    uint64_t n_inv = oracle_powmod((uint64_t)(n % q), q - 2, q);
    uint64_t p = n_inv;
    for (size_t i = 0; i < n; i++) {
        a[i] = oracle_mulmod(a[i], p, q);
        p = oracle_mulmod(p, psi_inv, q);
    }
}

/*
 * count independent negacyclic products c[r] = a[r] * b[r] mod (X^n + 1, q[r]),
 * each row of n residues; psi[r] is a primitive 2n-th root of unity mod q[r].
 */
void oracle_polymul_batch(const uint64_t *a, const uint64_t *b, uint64_t *c, size_t count,
                          size_t n, const uint64_t *q, const uint64_t *psi)
{
    #pragma omp parallel for schedule(dynamic)
    for (long r = 0; r < (long)count; r++) {
        uint64_t *fa = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *fb = (uint64_t *)malloc(n * sizeof(uint64_t));
        memcpy(fa, a + (size_t)r * n, n * sizeof(uint64_t));
        memcpy(fb, b + (size_t)r * n, n * sizeof(uint64_t));
        oracle_ntt_negacyclic(fa, n, q[r], psi[r]);
        oracle_ntt_negacyclic(fb, n, q[r], psi[r]);
        for (size_t i = 0; i < n; i++) fa[i] = oracle_mulmod(fa[i], fb[i], q[r]);
        oracle_intt_negacyclic(fa, n, q[r], psi[r]);
        memcpy(c + (size_t)r * n, fa, n * sizeof(uint64_t));
        free(fa);
        free(fb);
    }
}

/* count independent forward (inverse != 0: inverse) transforms, in place. */
void oracle_ntt_batch(uint64_t *a, size_t count, size_t n, const uint64_t *q,
                      const uint64_t *psi, int inverse)
{
    #pragma omp parallel for schedule(dynamic)
    for (long r = 0; r < (long)count; r++) {
        if (inverse) oracle_intt_negacyclic(a + (size_t)r * n, n, q[r], psi[r]);
        else oracle_ntt_negacyclic(a + (size_t)r * n, n, q[r], psi[r]);
    }
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
