/*
 * Device building blocks shared by every run-time compiled kernel (gfx950,
 * wave64).  This text is prepended to each generated kernel source; the
 * generator adds the tree's element function and the kernel bodies.
 *
 * Floating-point rules: no contraction (a*b+c stays two rounded operations
 * unless fmaf/fma is written on purpose), IEEE divide and square root
 * (correctly rounded), denormals kept, no fast-math.
 */
#pragma clang fp contract(off)

typedef unsigned short u16;
typedef unsigned int u32;
typedef unsigned long long u64;
typedef long long i64;
typedef u32 u32x4 __attribute__((ext_vector_type(4)));
typedef u32 u32x2 __attribute__((ext_vector_type(2)));

#define CD __device__ __forceinline__

/* ------------------------------------------------------------------ */
/* storage <-> compute conversions                                     */
/* ------------------------------------------------------------------ */
/* 16-bit storage widens exactly to FP32. */
CD float widen_bf16(u16 b) { return __builtin_bit_cast(float, (u32)b << 16); }
CD float widen_f16(u16 b) { return (float)__builtin_bit_cast(_Float16, b); }

/* FP32 -> bfloat16 bits, round to nearest even; NaN stays a quiet NaN. */
CD u16 bits_bf16(float f)
{
    u32 u = __builtin_bit_cast(u32, f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
/* FP32 -> binary16 bits: the hardware conversion rounds to nearest even. */
CD u16 bits_f16(float f) { return __builtin_bit_cast(u16, (_Float16)f); }

/* FP64 -> FP32 rounded to odd (truncate, then set the last bit if inexact).
 * Rounding to odd into a format with at least two more bits than the final
 * 16-bit format makes the following round-to-nearest-even exact
 * (Boldo and Melquiond, "Emulation of FMA and correctly rounded sums: proved
 * algorithms using rounding to odd", IEEE Trans. Computers 57(4), 2008). */
CD float f32_round_odd(double d)
{
    float f = (float)d;
    if ((double)f != d && d == d) {
        u32 u = __builtin_bit_cast(u32, f);
        if (__builtin_fabs((double)f) > __builtin_fabs(d)) u -= 1u;  /* step toward zero */
        u |= 1u;
        f = __builtin_bit_cast(float, u);
    }
    return f;
}
CD u16 bits_bf16_d(double d) { return bits_bf16(f32_round_odd(d)); }
CD u16 bits_f16_d(double d) { return bits_f16(f32_round_odd(d)); }

/* value of a number after rounding to a 16-bit type (used by conv nodes) */
CD float rnd_bf16(float f) { return widen_bf16(bits_bf16(f)); }
CD float rnd_f16(float f) { return widen_f16(bits_f16(f)); }
CD float rnd_bf16_d(double d) { return widen_bf16(bits_bf16_d(d)); }
CD float rnd_f16_d(double d) { return widen_f16(bits_f16_d(d)); }

/* FP64 -> 32-bit integer: the fraction dropped toward zero, the result
 * clamped to the type's range, NaN -> 0 */
CD int sat_i32(double x)
{
    if (x != x) return 0;
    x = __builtin_trunc(x);
    return x <= -2147483648.0 ? (int)0x80000000u : (x >= 2147483647.0 ? 0x7fffffff : (int)x);
}
CD unsigned sat_u32(double x)
{
    if (x != x) return 0u;
    x = __builtin_trunc(x);
    return x <= 0.0 ? 0u : (x >= 4294967295.0 ? 0xffffffffu : (unsigned)x);
}

/* ------------------------------------------------------------------ */
/* vector loads / stores of VE consecutive elements                     */
/* ------------------------------------------------------------------ */
template <int BYTES> struct rawvec;
template <> struct rawvec<16> { typedef u32x4 T; };
template <> struct rawvec<8> { typedef u32x2 T; };
template <> struct rawvec<4> { typedef u32 T; };
template <> struct rawvec<2> { typedef u16 T; };

/* Streaming data is touched once: loads and stores carry the nontemporal
 * hint, which measurably raises HBM throughput on gfx950 for streams larger
 * than the caches. */
#ifndef COOT_NT
#define COOT_NT 1
#endif

template <class S, int VE>
CD void ldv(const S* __restrict__ p, i64 e0, S (&o)[VE])
{
    constexpr int B = (int)sizeof(S) * VE;
    if constexpr (B <= 16) {
        typedef typename rawvec<B>::T R;
#if COOT_NT
        R r = __builtin_nontemporal_load((const R*)(p + e0));
#else
        R r = *(const R*)(p + e0);
#endif
        __builtin_memcpy(o, &r, B);
    } else {
        ldv<S, VE / 2>(p, e0, *(S(*)[VE / 2])o);
        ldv<S, VE / 2>(p, e0 + VE / 2, *(S(*)[VE / 2])(o + VE / 2));
    }
}

template <class S, int VE>
CD void stv(S* p, i64 e0, const S (&o)[VE])
{
    constexpr int B = (int)sizeof(S) * VE;
    if constexpr (B <= 16) {
        typedef typename rawvec<B>::T R;
        R r;
        __builtin_memcpy(&r, o, B);
#if COOT_NT
        __builtin_nontemporal_store(r, (R*)(p + e0));
#else
        *(R*)(p + e0) = r;
#endif
    } else {
        stv<S, VE / 2>(p, e0, *(const S(*)[VE / 2])o);
        stv<S, VE / 2>(p, e0 + VE / 2, *(const S(*)[VE / 2])(o + VE / 2));
    }
}

/* VE consecutive elements to / from LDS in one access (e0 a multiple of VE) */
template <class S, int VE>
CD void lds_put(S* p, int e0, const S (&o)[VE])
{
    typedef typename rawvec<(int)sizeof(S) * VE>::T R;
    R r;
    __builtin_memcpy(&r, o, sizeof r);
    *(R*)(p + e0) = r;
}

template <class S, int VE>
CD void lds_get(const S* p, int e0, S (&o)[VE])
{
    typedef typename rawvec<(int)sizeof(S) * VE>::T R;
    const R r = *(const R*)(p + e0);
    __builtin_memcpy(o, &r, sizeof r);
}

/* order the LDS accesses of one wave's lanes (LDS instructions of a wave
 * complete in order; this keeps the compiler from moving them) */
CD void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

/* single-element streaming load / store */
template <class S>
CD S ldnt(const S* p)
{
#if COOT_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

template <class S>
CD void stnt(S* p, S v)
{
#if COOT_NT
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

/* element at a 32-bit element offset from a base (the byte offset is formed
 * in 32 bits, so the access takes a scalar base and a vector offset) */
template <class S>
CD const S* at(const S* base, u32 off)
{
    return (const S*)((const char*)base + off * (u32)sizeof(S));
}

template <class S>
CD S* atw(S* base, u32 off)
{
    return (S*)((char*)base + off * (u32)sizeof(S));
}

/* single-element load / store through the caches */
template <class S>
CD S ldpl(const S* p)
{
    return *p;
}

template <class S>
CD void stpl(S* p, S v)
{
    *p = v;
}

/* ------------------------------------------------------------------ */
/* accumulators                                                         */
/* ------------------------------------------------------------------ */
/* Compensated FP32 sum: (s, c) with every step an exact TwoSum (Knuth) and
 * products split exactly with TwoProduct (fmaf).  The value is s + c. */
struct AccKF {
    float s, c;
    CD void init() { s = 0.0f; c = 0.0f; }
    CD void add(float x)
    {
        float t = s + x;
        float z = t - s;
        c += (s - (t - z)) + (x - z);
        s = t;
    }
    CD void add_prod(float a, float b)
    {
        float p = a * b;
        float e = __builtin_fmaf(a, b, -p);
        add(p);
        c += e;
    }
    CD void merge(const AccKF& o)
    {
        float t = s + o.s;
        float z = t - s;
        float e = (s - (t - z)) + (o.s - z);
        s = t;
        c = (c + o.c) + e;
    }
    CD void shfl(int off)
    {
        AccKF o;
        o.s = __shfl_xor(s, off, 64);
        o.c = __shfl_xor(c, off, 64);
        merge(o);
    }
    CD double hi() const { return (double)s; }
    /* Once the sum is infinite or NaN every later TwoSum makes c NaN; the
     * value is then s alone (inf + finite = inf, inf + -inf = NaN, as in
     * IEEE addition). */
    CD double lo() const { return __builtin_isfinite(s) ? (double)c : 0.0; }
};

/* Plain FP32 sum (the "pairwise only" variant: per-thread running sum, then
 * the same binary trees with no compensation). */
struct AccPF {
    float s;
    CD void init() { s = 0.0f; }
    CD void add(float x) { s += x; }
    CD void add_prod(float a, float b) { s += a * b; }
    CD void merge(const AccPF& o) { s = s + o.s; }
    CD void shfl(int off)
    {
        AccPF o;
        o.s = __shfl_xor(s, off, 64);
        merge(o);
    }
    CD double hi() const { return (double)s; }
    CD double lo() const { return 0.0; }
};

/* Compensated FP64 sum (F64 data, and the cross-block combine). */
struct AccKD {
    double s, c;
    CD void init() { s = 0.0; c = 0.0; }
    CD void add(double x)
    {
        double t = s + x;
        double z = t - s;
        c += (s - (t - z)) + (x - z);
        s = t;
    }
    CD void add_prod(double a, double b)
    {
        double p = a * b;
        double e = __builtin_fma(a, b, -p);
        add(p);
        c += e;
    }
    CD void merge(const AccKD& o)
    {
        double t = s + o.s;
        double z = t - s;
        double e = (s - (t - z)) + (o.s - z);
        s = t;
        c = (c + o.c) + e;
    }
    CD void shfl(int off)
    {
        AccKD o;
        o.s = __shfl_xor(s, off, 64);
        o.c = __shfl_xor(c, off, 64);
        merge(o);
    }
    CD double hi() const { return s; }
    CD double lo() const { return __builtin_isfinite(s) ? c : 0.0; }  // as AccKF::lo
};

/* Variance accumulator, FP64 for every storage type: the count c, a shift k
 * (the first value seen) and the sums of x - k and (x - k)^2, so that the
 * cancellation in sum((x - mean)^2) is that of values near k.  Two states
 * merge pairwise (Chan, Golub and LeVeque, "Updating formulae and a pairwise
 * algorithm for computing sample variances", 1979): each is read as
 * (count, mean, M2) and the merged state keeps its mean as the shift.  A NaN
 * value propagates. */
struct AccV {
    double c, k, s, q;
    CD void init() { c = 0.0; k = 0.0; s = 0.0; q = 0.0; }
    CD void add(double x)
    {
        k = c == 0.0 ? x : k;
        const double d = x - k;
        s += d;
        q += d * d;
        c += 1.0;
    }
    CD double mean() const { return k + s / c; }
    CD double m2() const
    {
        const double m = q - s * (s / c);
        return m < 0.0 ? 0.0 : m;
    }
    CD void merge(const AccV& o)
    {
        if (o.c == 0.0) return;
        if (c == 0.0) {
            *this = o;
            return;
        }
        const double n = c + o.c, ma = mean(), mb = o.mean(), d = mb - ma;
        const double M = (m2() + o.m2()) + d * d * (c * o.c / n);
        k = ma + d * (o.c / n);
        s = 0.0;
        q = M;
        c = n;
    }
    CD void shfl(int off)
    {
        AccV o;
        o.c = __shfl_xor(c, off, 64);
        o.k = __shfl_xor(k, off, 64);
        o.s = __shfl_xor(s, off, 64);
        o.q = __shfl_xor(q, off, 64);
        merge(o);
    }
    /* unbiased (n - 1) variance; 0 for one value, NaN for none */
    CD double var() const
    {
        if (c == 0.0) return __builtin_nan("");
        if (c < 2.0) return 0.0;
        return m2() / (c - 1.0);
    }
};

/* Extremum with its index: NaN skipped, ties to the lowest index, i < 0
 * means "nothing seen yet". */
template <class C, bool MAX>
struct AccI {
    C v;
    i64 i;
    CD void init() { v = (C)0; i = -1; }
    /* selections are written as selects, not branches: a per-element
     * branch costs more than the compares it guards */
    CD bool better(C x, i64 j) const
    {
        const bool gt = MAX ? (x > v) : (x < v);
        return (i < 0) | gt | ((x == v) & (j < i));
    }
    CD void add(C x, i64 j)
    {
        const bool t = (x == x) & better(x, j);
        v = t ? x : v;
        i = t ? j : i;
    }
    /* the same for a stream whose indices only grow (j above every index
     * seen so far): a tie never replaces the earlier element */
    CD void add_inc(C x, i64 j)
    {
        const bool t = (x == x) & ((i < 0) | (MAX ? (x > v) : (x < v)));
        v = t ? x : v;
        i = t ? j : i;
    }
    CD void merge(const AccI& o)
    {
        const bool t = (o.i >= 0) & better(o.v, o.i);
        v = t ? o.v : v;
        i = t ? o.i : i;
    }
    CD void shfl(int off)
    {
        AccI o;
        o.v = __shfl_xor(v, off, 64);
        o.i = __shfl_xor(i, off, 64);
        merge(o);
    }
};

/* ------------------------------------------------------------------ */
/* wave64 and block reductions (fixed order: deterministic)             */
/* ------------------------------------------------------------------ */
template <class A>
CD void wave_reduce(A& a)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) a.shfl(off);
}

/* Result valid in thread 0.  lds must hold blockDim.x/64 entries. */
template <class A>
CD A block_reduce(A a, A* lds)
{
    wave_reduce(a);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) lds[w] = a;
    __syncthreads();
    if (w == 0) {
        A b;
        if (lane < nw) b = lds[lane];
        else b.init();
        wave_reduce(b);
        a = b;
    }
    return a;
}

/* partial slots are 16 bytes: sums (hi, lo) as two doubles; extrema
 * (value as double, index). */
CD void put_sum_partial(double* part, i64 slot, double hi, double lo)
{
    part[2 * slot] = hi;
    part[2 * slot + 1] = lo;
}

CD void put_idx_partial(double* part, i64 slot, double v, i64 i)
{
    part[2 * slot] = v;
    part[2 * slot + 1] = __builtin_bit_cast(double, i);
}

/* variance partials: 4 doubles per slot */
CD void put_var_partial(double* part, i64 slot, const AccV& a)
{
    double* p = part + 4 * slot;
    p[0] = a.c;
    p[1] = a.k;
    p[2] = a.s;
    p[3] = a.q;
}

CD AccV var_partial(const double* part, i64 slot)
{
    const double* p = part + 4 * slot;
    AccV a;
    a.c = p[0];
    a.k = p[1];
    a.s = p[2];
    a.q = p[3];
    return a;
}

/* merge `count` variance partials (first, stride) in a fixed order */
CD AccV combine_var(const double* part, i64 first, i64 count, i64 stride)
{
    __shared__ AccV lds_v[16];
    AccV a;
    a.init();
    const i64 bd = blockDim.x;
    for (i64 t = threadIdx.x; t < count; t += 4 * bd) {
        AccV o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const i64 tu = t + u * bd;
            o[u] = var_partial(part, first + (tu < count ? tu : t) * stride);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t + u * bd < count) a.merge(o[u]);
    }
    return block_reduce(a, lds_v);
}

CD AccV combine_var_seq(const double* part, i64 first, i64 count, i64 stride)
{
    AccV a;
    a.init();
    for (i64 t = 0; t < count; t += 4) {
        AccV o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) o[u] = var_partial(part, first + (t + u < count ? t + u : t) * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t + u < count) a.merge(o[u]);
    }
    return a;
}

/* FP64 compensated combine of `count` sum partials starting at `first`,
 * with `stride` doubles-pairs between them; result in thread 0. */
CD double combine_sums(const double* part, i64 first, i64 count, i64 stride)
{
    __shared__ AccKD lds_kd[16];
    AccKD a;
    a.init();
    // four partials per thread are loaded before any is added (one memory
    // latency instead of four); the thread still adds them in index order
    const i64 bd = blockDim.x;
    for (i64 t = threadIdx.x; t < count; t += 4 * bd) {
        double h[4], l[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const i64 tu = t + u * bd;
            const double* p = part + 2 * (first + (tu < count ? tu : t) * stride);
            h[u] = p[0];
            l[u] = p[1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t + u * bd < count) {
                a.add(h[u]);
                a.add(l[u]);
            }
    }
    a = block_reduce(a, lds_kd);
    return a.hi() + a.lo();
}

template <bool MAX>
CD AccI<double, MAX> combine_idx(const double* part, i64 first, i64 count, i64 stride)
{
    __shared__ AccI<double, MAX> lds_id[16];
    AccI<double, MAX> a;
    a.init();
    const i64 bd = blockDim.x;
    for (i64 t = threadIdx.x; t < count; t += 4 * bd) {
        AccI<double, MAX> o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const i64 tu = t + u * bd;
            const double* p = part + 2 * (first + (tu < count ? tu : t) * stride);
            o[u].v = p[0];
            o[u].i = __builtin_bit_cast(i64, p[1]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t + u * bd < count) a.merge(o[u]);
    }
    return block_reduce(a, lds_id);
}

/* the same combines done by one thread, partials in order */
CD double combine_sums_seq(const double* part, i64 first, i64 count, i64 stride)
{
    AccKD a;
    a.init();
    // eight partials are loaded before any is added; the adds keep index order
    for (i64 t = 0; t < count; t += 8) {
        double h[8], l[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double* p = part + 2 * (first + (t + u < count ? t + u : t) * stride);
            h[u] = p[0];
            l[u] = p[1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (t + u < count) {
                a.add(h[u]);
                a.add(l[u]);
            }
    }
    return a.hi() + a.lo();
}

template <bool MAX>
CD AccI<double, MAX> combine_idx_seq(const double* part, i64 first, i64 count, i64 stride)
{
    AccI<double, MAX> a;
    a.init();
    for (i64 t = 0; t < count; t += 8) {
        AccI<double, MAX> o[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double* p = part + 2 * (first + (t + u < count ? t + u : t) * stride);
            o[u].v = p[0];
            o[u].i = __builtin_bit_cast(i64, p[1]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (t + u < count) a.merge(o[u]);
    }
    return a;
}

/* write a reduction value / index to the output buffer */
CD void put_f32(void* out, i64 j, double v) { ((float*)out)[j] = (float)v; }
CD void put_f64(void* out, i64 j, double v) { ((double*)out)[j] = v; }
CD void put_u64(void* out, i64 j, i64 i) { ((u64*)out)[j] = (u64)(i < 0 ? 0 : i); }
