/*
 * lsb_oracle.c -- plain, bit-by-bit CPU oracle (see lsb_oracle.h).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Written for a reader who checks it
 * against the paper by eye: one stream bit at a time, no blocking, no tables.
 *
 * Paper passages followed:
 *   Section VI step 7 (embedding): per cover byte, keep the bits outside the
 *     field (the paper's mask 1111 1100), OR in the data bits (its masks
 *     0000 0011 .. 1100 0000 shifted right by 2i).  Generalised to k bits.
 *   Section VI step 5 / Section VII step 4: the data must fit; at 2 bits per
 *     cover byte one data byte needs 4 cover bytes, i.e. n*k/8 stream bytes
 *     fit an n-byte cover in general.
 *   Section VII step 6 (extraction): mask the field (0000 0011), shift it to
 *     its place in the data byte and OR it into the zero-initialised byte.
 * Readings (paper silent): MSB-first stream, BE32 length header, sequential
 * placement over every channel byte, partial last field keeps the cover's
 * remaining low bits, bytes past the stream unchanged.
 */
#include "lsb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Bit j of a byte string read most-significant bit first. */
static unsigned get_bit(const uint8_t *bytes, uint64_t j)
{
    return (bytes[j / 8] >> (7 - (j % 8))) & 1u;
}

static void set_bit(uint8_t *bytes, uint64_t j, unsigned bit)
{
    if (bit)
        bytes[j / 8] |= (uint8_t)(0x80u >> (j % 8));
}

/* floor(n*k/8) without overflowing 64 bits. */
static uint64_t bits_to_bytes_floor(uint64_t n, int k)
{
    return (n / 8) * (uint64_t)k + ((n % 8) * (uint64_t)k) / 8;
}

int64_t oracle_capacity(uint64_t n, int k)
{
    if (k < 1 || k > 8)
        return ORACLE_E_ARG;
    uint64_t room = bits_to_bytes_floor(n, k); /* whole stream bytes that fit */
    if (room < 4)
        return ORACLE_E_CAPACITY;
    uint64_t cap = room - 4;
    if (cap > 0xFFFFFFFFull)
        cap = 0xFFFFFFFFull;
    return (int64_t)cap;
}

int oracle_embed_raw(const uint8_t *cover, uint8_t *stego, uint64_t n,
                     uint64_t t0, const uint8_t *stream, uint64_t stream_bits,
                     int k)
{
    if (k < 1 || k > 8)
        return ORACLE_E_ARG;
    if (n > 0 && (!cover || !stego))
        return ORACLE_E_ARG;
    if (stream_bits > 0 && !stream)
        return ORACLE_E_ARG;

    for (uint64_t t = 0; t < n; ++t) {
        uint64_t first = (uint64_t)k * (t0 + t); /* first stream bit of field */
        if (first >= stream_bits) {
            stego[t] = cover[t]; /* past the stream: unchanged */
            continue;
        }
        uint64_t left = stream_bits - first;
        unsigned nb = left < (uint64_t)k ? (unsigned)left : (unsigned)k;
        /* v = the nb stream bits, first bit most significant */
        unsigned v = 0;
        for (unsigned q = 0; q < nb; ++q)
            v = (v << 1) | get_bit(stream, first + q);
        /* the nb bits occupy the top of the k-bit field */
        unsigned shift = (unsigned)k - nb;
        unsigned mask = ((1u << nb) - 1u) << shift;
        stego[t] = (uint8_t)((cover[t] & ~mask & 0xFFu) | (v << shift));
    }
    return ORACLE_OK;
}

int oracle_extract_raw(const uint8_t *stego, uint64_t n, uint64_t t0,
                       uint8_t *stream_out, uint64_t stream_bits, int k)
{
    if (k < 1 || k > 8)
        return ORACLE_E_ARG;
    uint64_t begin = (uint64_t)k * t0;
    uint64_t end = (uint64_t)k * (t0 + n);
    if (end > stream_bits)
        end = stream_bits;
    if (begin % 8 != 0)
        return ORACLE_E_ARG;
    if (begin >= end)
        return ORACLE_OK; /* this slice carries no stream bits */
    if (end % 8 != 0 && end != stream_bits)
        return ORACLE_E_ARG;
    if (!stego || !stream_out)
        return ORACLE_E_ARG;

    /* zero-initialise the output bytes (Section VII step 4), then OR bits in */
    uint64_t first_byte = begin / 8;
    uint64_t last_byte = (end + 7) / 8; /* exclusive */
    memset(stream_out + first_byte, 0, (size_t)(last_byte - first_byte));
    for (uint64_t j = begin; j < end; ++j) {
        uint64_t t = j / (uint64_t)k - t0; /* field holding stream bit j */
        unsigned q = (unsigned)(j % (uint64_t)k); /* its place in the field */
        unsigned bit = (stego[t] >> ((unsigned)k - 1 - q)) & 1u;
        set_bit(stream_out, j, bit);
    }
    return ORACLE_OK;
}

int oracle_embed(const uint8_t *cover, uint8_t *stego, uint64_t n,
                 const uint8_t *msg, uint32_t len, int k)
{
    int64_t cap = oracle_capacity(n, k);
    if (cap < 0)
        return (int)cap;
    if ((uint64_t)len > (uint64_t)cap)
        return ORACLE_E_CAPACITY;
    if (len > 0 && !msg)
        return ORACLE_E_ARG;

    /* S = BE32(len) || msg, assembled explicitly */
    uint64_t s_bytes = 4 + (uint64_t)len;
    uint8_t *s = (uint8_t *)malloc((size_t)s_bytes);
    if (!s)
        return ORACLE_E_NOMEM;
    s[0] = (uint8_t)(len >> 24);
    s[1] = (uint8_t)(len >> 16);
    s[2] = (uint8_t)(len >> 8);
    s[3] = (uint8_t)len;
    if (len > 0)
        memcpy(s + 4, msg, len);
    int rc = oracle_embed_raw(cover, stego, n, 0, s, 8 * s_bytes, k);
    free(s);
    return rc;
}

int oracle_extract(const uint8_t *stego, uint64_t n, int k,
                   uint8_t *msg_out, uint64_t out_cap, uint32_t *len_out)
{
    if (k < 1 || k > 8 || !len_out)
        return ORACLE_E_ARG;
    *len_out = 0;
    uint64_t cover_bits = (uint64_t)k * n;
    if (cover_bits < 32)
        return ORACLE_E_HEADER; /* not even the header fits */

    /* header: stream bits 0..31, a big-endian byte count */
    uint8_t hdr[4];
    int rc = oracle_extract_raw(stego, n, 0, hdr, 32, k);
    if (rc != ORACLE_OK)
        return rc;
    uint32_t len = ((uint32_t)hdr[0] << 24) | ((uint32_t)hdr[1] << 16) |
                   ((uint32_t)hdr[2] << 8) | (uint32_t)hdr[3];
    *len_out = len;
    if (4 + (uint64_t)len > bits_to_bytes_floor(n, k))
        return ORACLE_E_HEADER;
    if ((uint64_t)len > out_cap)
        return ORACLE_E_BUFFER;
    if (len == 0)
        return ORACLE_OK;
    if (!msg_out)
        return ORACLE_E_ARG;

    uint64_t s_bytes = 4 + (uint64_t)len;
    uint8_t *s = (uint8_t *)malloc((size_t)s_bytes);
    if (!s)
        return ORACLE_E_NOMEM;
    rc = oracle_extract_raw(stego, n, 0, s, 8 * s_bytes, k);
    if (rc == ORACLE_OK)
        memcpy(msg_out, s + 4, len);
    free(s);
    return rc;
}

/* ------------------------------------------------------------------------
 * The paper's own layout.  Section VI: separate one plane (step 2), give
 * each row a data chunk B with size(B)*4 <= size(A) (steps 4-5), and for
 * block i = 0..3 and thread j = 0..L-1 take bits 2i+1..2i of B[j] (mask
 * 0000 0011 << 2i, then shift right by 2i) into pixel A[L*i + j], whose low
 * two bits are cleared with 1111 1100 (step 7).  Section VII: B starts at
 * zero (step 4); for each i, j the low two bits of A[L*i + j], shifted left
 * by 2i, are ORed into B[j] (step 6).
 */
uint64_t oracle_paper_capacity(uint32_t h, uint32_t w)
{
    return (uint64_t)h * (w / 4);
}

/* pixel x of row y of the plane */
static uint64_t plane_index(uint32_t y, uint32_t x, uint32_t w, uint32_t c,
                            uint32_t plane)
{
    return ((uint64_t)y * w + x) * c + plane;
}

int oracle_paper_embed(const uint8_t *cover, uint8_t *stego, uint32_t h,
                       uint32_t w, uint32_t c, uint32_t plane,
                       const uint8_t *data, uint64_t len)
{
    if (c == 0 || plane >= c)
        return ORACLE_E_ARG;
    if (len > oracle_paper_capacity(h, w))
        return ORACLE_E_CAPACITY;
    uint64_t n = (uint64_t)h * w * c;
    if (n > 0 && (!cover || !stego))
        return ORACLE_E_ARG;
    if (len > 0 && !data)
        return ORACLE_E_ARG;
    if (stego != cover)
        memcpy(stego, cover, (size_t)n);

    uint64_t remaining = len, off = 0;
    for (uint32_t y = 0; y < h && remaining > 0; ++y) {
        uint64_t L = remaining < w / 4 ? remaining : w / 4; /* size(B) */
        const uint8_t *B = data + off;
        for (unsigned i = 0; i < 4; ++i) {
            for (uint64_t j = 0; j < L; ++j) {
                unsigned v = B[j];
                v &= 3u << (2 * i);
                v >>= 2 * i;
                uint64_t at = plane_index(y, (uint32_t)(L * i + j), w, c, plane);
                stego[at] = (uint8_t)((stego[at] & 0xFCu) | v);
            }
        }
        off += L;
        remaining -= L;
    }
    return ORACLE_OK;
}

int oracle_paper_extract(const uint8_t *stego, uint32_t h, uint32_t w,
                         uint32_t c, uint32_t plane, uint8_t *data,
                         uint64_t len)
{
    if (c == 0 || plane >= c)
        return ORACLE_E_ARG;
    if (len > oracle_paper_capacity(h, w))
        return ORACLE_E_CAPACITY;
    if (len > 0 && (!stego || !data))
        return ORACLE_E_ARG;

    uint64_t remaining = len, off = 0;
    for (uint32_t y = 0; y < h && remaining > 0; ++y) {
        uint64_t L = remaining < w / 4 ? remaining : w / 4;
        uint8_t *B = data + off;
        memset(B, 0, (size_t)L);
        for (unsigned i = 0; i < 4; ++i) {
            for (uint64_t j = 0; j < L; ++j) {
                uint64_t at = plane_index(y, (uint32_t)(L * i + j), w, c, plane);
                unsigned v = stego[at] & 3u;
                v <<= 2 * i;
                B[j] = (uint8_t)(B[j] | v);
            }
        }
        off += L;
        remaining -= L;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * One colour plane with the general method: gather the plane (Section VI
 * step 2), run the plain definition on it, scatter it back.
 */
int oracle_embed_plane(const uint8_t *cover, uint8_t *stego, uint64_t pixels,
                       uint32_t c, uint32_t plane, const uint8_t *msg,
                       uint32_t len, int k)
{
    if (c == 0 || plane >= c || (pixels > 0 && (!cover || !stego)))
        return ORACLE_E_ARG;
    int64_t cap = oracle_capacity(pixels, k);
    if (cap < 0)
        return (int)cap;
    if ((uint64_t)len > (uint64_t)cap)
        return ORACLE_E_CAPACITY;
    uint8_t *a = (uint8_t *)malloc(pixels ? (size_t)pixels : 1);
    uint8_t *b = (uint8_t *)malloc(pixels ? (size_t)pixels : 1);
    if (!a || !b) {
        free(a);
        free(b);
        return ORACLE_E_NOMEM;
    }
    for (uint64_t p = 0; p < pixels; ++p)
        a[p] = cover[p * c + plane];
    int rc = oracle_embed(a, b, pixels, msg, len, k);
    if (rc == ORACLE_OK) {
        if (stego != cover)
            memcpy(stego, cover, (size_t)(pixels * c));
        for (uint64_t p = 0; p < pixels; ++p)
            stego[p * c + plane] = b[p];
    }
    free(a);
    free(b);
    return rc;
}

int oracle_extract_plane(const uint8_t *stego, uint64_t pixels, uint32_t c,
                         uint32_t plane, int k, uint8_t *msg_out,
                         uint64_t out_cap, uint32_t *len_out)
{
    if (c == 0 || plane >= c || !len_out || (pixels > 0 && !stego))
        return ORACLE_E_ARG;
    uint8_t *a = (uint8_t *)malloc(pixels ? (size_t)pixels : 1);
    if (!a)
        return ORACLE_E_NOMEM;
    for (uint64_t p = 0; p < pixels; ++p)
        a[p] = stego[p * c + plane];
    int rc = oracle_extract(a, pixels, k, msg_out, out_cap, len_out);
    free(a);
    return rc;
}

uint64_t oracle_sse(const uint8_t *a, const uint8_t *b, uint64_t n)
{
    uint64_t sum = 0;
    for (uint64_t i = 0; i < n; ++i) {
        int64_t d = (int64_t)a[i] - (int64_t)b[i];
        sum += (uint64_t)(d * d);
    }
    return sum;
}

double oracle_psnr(uint64_t sse, uint64_t count)
{
    if (sse == 0 || count == 0)
        return INFINITY;
    double mse = (double)sse / (double)count;
    return 10.0 * log10(255.0 * 255.0 / mse);
}
