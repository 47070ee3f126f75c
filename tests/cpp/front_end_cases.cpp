// Test cases of the C++ front end (include/coot.hpp): each entry point runs
// one group of front-end expressions on device memory the caller (the Python
// GPU tests, through ctypes) owns, so that the results can be compared with
// the CPU oracle.  Every function returns 0, or -1 with the exception's
// message in fe_last_error().  `stream` is the caller's HIP stream.
#include <cstdio>
#include <cstring>
#include <string>

#include "coot.hpp"

using namespace coot;

static thread_local std::string g_err;

template <class F>
static int guard(void* stream, F&& f)
{
    try {
        set_stream((hipStream_t)stream);
        f();
        synchronise();
        return 0;
    } catch (const std::exception& e) {
        g_err = e.what();
        return -1;
    }
}

extern "C" {

const char* fe_last_error(void) { return g_err.c_str(); }

// Y = 2.5*A + B%C - exp(D); s = accu(A % B); colsum = sum(A, 0);
// idx = index_max(abs(B)) -- the small plain-method workload
int fe_small(float* A, float* B, float* C, float* D, float* Y, int64_t r, int64_t c, float* colsum, float* s,
             uint64_t* idx, void* stream)
{
    return guard(stream, [&] {
        fmat a(A, r, c), b(B, r, c), cc(C, r, c), d(D, r, c), y(Y, r, c);
        y = 2.5 * a + b % cc - exp(d);
        *s = accu(a % b);
        fmat cs(colsum, 1, c);
        cs = sum(a, 0);
        *idx = index_max(abs(b));
    });
}

// in-place updates: A = trans(A) + 1 (the transposed read of the destination
// goes through a temporary); B += A; B %= A; B *= 0.5; B -= 1
int fe_in_place(float* A, float* B, int64_t n, void* stream)
{
    return guard(stream, [&] {
        fmat a(A, n, n), b(B, n, n);
        a = trans(a) + 1.0;
        b += a;
        b %= a;
        b *= 0.5;
        b -= 1.0;
    });
}

// views on an r x c FP64 matrix: A.diag() += 1; A.submat(1,1,3,3) = 2 *
// A.submat(0,0,2,2) (overlapping: the right side is evaluated first);
// A.row(r-1) = A.row(0) - A.row(1); A.col(c-1).fill(7); t = trace(A);
// dv = diagvec(A, k)
int fe_views(double* A, int64_t r, int64_t c, int64_t k, double* dv, int64_t nd, double* t, void* stream)
{
    return guard(stream, [&] {
        mat a(A, r, c);
        a.diag() += 1.0;
        a.submat(1, 1, 3, 3) = 2.0 * a.submat(0, 0, 2, 2);
        a.row(r - 1) = a.row(0) - a.row(1);
        a.col(c - 1).fill(7.0);
        *t = trace(a);
        vec d(dv, nd);
        d = diagvec(a, k);
    });
}

// generators: Y = 3*eye + ones + trans(eye(c, r)); L = linspace(a, b, n);
// Z.eye() on an owned matrix, copied back to host H (r x c)
int fe_generators(float* Y, int64_t r, int64_t c, double* L, int64_t n, double a, double b, float* H, void* stream)
{
    return guard(stream, [&] {
        fmat y(Y, r, c);
        y = 3.0 * eye<fmat>(r, c) + ones<fmat>(r, c) + trans(eye<fmat>(c, r));
        vec l(L, n);
        l = linspace<vec>(a, b, n);
        fmat z(r, c);
        z.eye();
        z.copy_to_host(H);
    });
}

// scalar-valued functions of FP64 vectors x, y (n elements): res[0..13]
int fe_scalars(double* X, double* Y, int64_t n, double* res, void* stream)
{
    return guard(stream, [&] {
        vec x(X, n), y(Y, n);
        res[0] = dot(x, y);
        res[1] = norm(x);
        res[2] = norm(x, 1);
        res[3] = norm(x, "inf");
        res[4] = norm(x, "-inf");
        res[5] = max(x);
        res[6] = min(x % y);
        res[7] = (double)index_min(x);
        res[8] = (double)index_max(x - y);
        res[9] = mean(x);
        res[10] = var(x);
        res[11] = accu(x > 0.3);
        res[12] = all(abs(x) < 100.0) ? 1.0 : 0.0;
        res[13] = any(x > 100.0) ? 1.0 : 0.0;
    });
}

// conversion fused into the kernel: F = conv_to<fmat>(2*X + 1) with X FP64;
// per-column and per-row statistics of F into cm (1 x c) and rv (r x 1)
int fe_convert(double* X, float* F, int64_t r, int64_t c, float* cm, float* rv, void* stream)
{
    return guard(stream, [&] {
        mat x(X, r, c);
        fmat f(F, r, c);
        f = conv_to<fmat>::from(2.0 * x + 1.0);
        fmat m(cm, 1, c), v(rv, r, 1);
        m = mean(f, 0);
        v = var(f, 1);
    });
}

// owned matrices: allocation, copy construction from an expression and from
// a matrix, move, host transfers; H (host, r x c) receives the result
int fe_owned(const float* Hin, int64_t r, int64_t c, float* H, void* stream)
{
    return guard(stream, [&] {
        fmat a(r, c);
        a.copy_from_host(Hin);
        fmat b = a * 2.0 + 1.0;
        fmat cc = b;
        fmat d(std::move(cc));
        d = d % a - trans(trans(a));
        d.copy_to_host(H);
    });
}

// 32-bit integer vectors a, b (n elements): F = conv_to<fvec>(2*a + b) fused;
// Q = a / b stored as integers (truncating division); U = a - b stored
// unsigned (negative values clamp to 0); s[0] = accu(a), s[1] = max(a % b)
int fe_integers(int32_t* A, int32_t* B, int64_t n, float* F, int32_t* Q, uint32_t* U, double* s, void* stream)
{
    return guard(stream, [&] {
        ivec a(A, n), b(B, n);
        fvec f(F, n);
        f = conv_to<fvec>::from(a * 2 + b);
        ivec q(Q, n);
        q = a / b;
        uvec u(U, n);
        u = conv_to<uvec>::from(a - b);
        s[0] = accu(a);
        s[1] = max(a % b);
    });
}

// an error crosses as an exception: adding matrices of different shapes
int fe_shape_error(float* A, float* B, void* stream)
{
    return guard(stream, [&] {
        fmat a(A, 4, 5), b(B, 5, 4), y(A, 4, 5);
        y = a + b;
    });
}

}  // extern "C"
