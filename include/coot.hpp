/* coot.hpp -- header-only C++17 front end over the C ABI of libcoot_mi355x.so.
 *
 * The Bandicoot paper (arXiv:2308.03120) presents its user interface as C++
 * expression templates (Section 7): every matrix, vector and expression
 * derives from Base<eT, Derived> (static polymorphism by the curiously
 * recurring template pattern), operators and functions return lightweight
 * expression objects (eOp, eGlue, Op<.., op_htrans>, mtOp) instead of
 * results, exact simplifications are chosen by overload resolution while the
 * expression type is built (trans(trans(X)) is X), and evaluation is delayed
 * until an assignment or a scalar-valued function.
 *
 * This header keeps that interface and replaces the evaluation: instead of
 * one kernel per node, an assignment flattens the expression type into the
 * postfix node array of coot.h and hands the whole tree to coot_eval, which
 * compiles it into one fused kernel; scalar functions (accu, dot, norm, min,
 * max, index_min, index_max, trace, all, any) call coot_reduce with a host
 * result.  Operands are column-major device matrices (Mat, Col, Row), views
 * (Table 1: .row, .col, .rows, .cols, .submat, .diag) and memory-free
 * generators (Table 4: eye, ones, zeros, linspace; Table 1 .fill/.ones/
 * .zeros/.eye).
 *
 * Lifetimes: an expression object holds references to the matrices it reads
 * and copies of its sub-expressions; like any expression template it is meant
 * to be used within the full expression that creates it (do not keep one in
 * an `auto` variable past the matrices it names).
 *
 * Errors: every library error becomes a std::runtime_error carrying
 * coot_last_error() (the paper's library reports errors by exception too).
 * Streams: all calls go to coot::get_stream() (default: the null stream).
 */
#ifndef COOT_HPP
#define COOT_HPP

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "coot.h"

namespace coot {

using uword = uint64_t;

// ---------------------------------------------------------------- runtime
inline void check(int rc)
{
    if (rc < 0) throw std::runtime_error(std::string("coot: ") + coot_last_error());
}

inline void check_hip(hipError_t e, const char* what)
{
    if (e != hipSuccess) throw std::runtime_error(std::string("coot: ") + what + ": " + hipGetErrorString(e));
}

inline hipStream_t& stream_slot()
{
    static thread_local hipStream_t s = nullptr;
    return s;
}
inline void set_stream(hipStream_t s) { stream_slot() = s; }
inline hipStream_t get_stream() { return stream_slot(); }
inline void synchronise() { check(coot_synchronise(get_stream())); }

template <class eT>
struct dtype_of;
template <>
struct dtype_of<float> {
    static constexpr int value = COOT_F32;
};
template <>
struct dtype_of<double> {
    static constexpr int value = COOT_F64;
};
template <>
struct dtype_of<int32_t> {
    static constexpr int value = COOT_I32;
};
template <>
struct dtype_of<uint32_t> {
    static constexpr int value = COOT_U32;
};

// type of a reduction's result: integer trees reduce in FP64 (exact sums
// below 2^53), floating-point trees in their own type
template <class eT>
using red_t = std::conditional_t<std::is_integral<eT>::value, double, eT>;

// ------------------------------------------------------- flattening context
// The postfix node array and operand table of one call.  A matrix read twice
// gets one operand slot (the library then reads it once).
struct Flat {
    std::vector<coot_node> nodes;
    std::vector<coot_operand> ops;
    std::vector<const void*> keys;

    int slot(const coot_operand& o, const void* key)
    {
        if (key)
            for (size_t i = 0; i < keys.size(); ++i)
                if (keys[i] == key && std::memcmp(&ops[i], &o, sizeof o) == 0) return (int)i;
        ops.push_back(o);
        keys.push_back(key);
        return (int)ops.size() - 1;
    }
    int push(int op, int a, int b, double k)
    {
        coot_node n;
        std::memset(&n, 0, sizeof n);
        n.op = op;
        n.a = a;
        n.b = b;
        n.k = k;
        nodes.push_back(n);
        return (int)nodes.size() - 1;
    }
    int leaf(const coot_operand& o, const void* key) { return push(COOT_LEAF, slot(o, key), -1, 0.0); }
    coot_expr expr() const
    {
        coot_expr e;
        std::memset(&e, 0, sizeof e);
        e.nodes = nodes.data();
        e.n_nodes = (int32_t)nodes.size();
        return e;
    }
};

// --------------------------------------------------------------- CRTP base
template <class eT, class Derived>
struct Base {
    using elem_type = eT;
    const Derived& get_ref() const { return static_cast<const Derived&>(*this); }
};

// Leaves (matrices) are held by reference, everything else by value.
template <class T>
struct is_leaf : std::false_type {};
template <class T>
using stored_t = std::conditional_t<is_leaf<T>::value, const T&, const T>;

template <class eT>
class Mat;
template <class eT>
class subview;

// ------------------------------------------------------------ expressions
// eOp: an element-wise unary or scalar node (k = the scalar)
template <class T1, int OP>
struct eOp : Base<typename T1::elem_type, eOp<T1, OP>> {
    stored_t<T1> m;
    double k;
    eOp(const T1& a, double kk = 0.0) : m(a), k(kk) {}
    int64_t n_rows() const { return m.n_rows(); }
    int64_t n_cols() const { return m.n_cols(); }
    int flatten(Flat& f) const { return f.push(OP, m.flatten(f), -1, k); }
};

// eGlue: an element-wise binary node
template <class T1, class T2, int OP>
struct eGlue : Base<typename T1::elem_type, eGlue<T1, T2, OP>> {
    stored_t<T1> a;
    stored_t<T2> b;
    eGlue(const T1& x, const T2& y) : a(x), b(y) {}
    int64_t n_rows() const { return a.n_rows(); }
    int64_t n_cols() const { return a.n_cols(); }
    int flatten(Flat& f) const
    {
        const int i = a.flatten(f);
        const int j = b.flatten(f);
        return f.push(OP, i, j, 0.0);
    }
};

struct op_htrans {};

// Op<T1, op_htrans>: the transpose, read in place by the fused kernel
template <class T1, class op_type>
struct Op : Base<typename T1::elem_type, Op<T1, op_type>> {
    stored_t<T1> m;
    explicit Op(const T1& a) : m(a) {}
    int64_t n_rows() const { return m.n_cols(); }
    int64_t n_cols() const { return m.n_rows(); }
    int flatten(Flat& f) const { return f.push(COOT_TRANS, m.flatten(f), -1, 0.0); }
};

// mtOp: conversion to another element type (fused into the kernel)
template <class out_eT, class T1>
struct mtOp : Base<out_eT, mtOp<out_eT, T1>> {
    stored_t<T1> m;
    explicit mtOp(const T1& a) : m(a) {}
    int64_t n_rows() const { return m.n_rows(); }
    int64_t n_cols() const { return m.n_cols(); }
    int flatten(Flat& f) const { return f.push(COOT_CONV, m.flatten(f), dtype_of<out_eT>::value, 0.0); }
};

// Gen: a memory-free generator leaf (Table 4)
template <class eT, uint32_t KIND>
struct Gen : Base<eT, Gen<eT, KIND>> {
    int64_t r, c;
    double g0, g1;
    Gen(int64_t rr, int64_t cc, double a = 0.0, double b = 0.0) : r(rr), c(cc), g0(a), g1(b) {}
    int64_t n_rows() const { return r; }
    int64_t n_cols() const { return c; }
    coot_operand operand() const
    {
        coot_operand o;
        std::memset(&o, 0, sizeof o);
        o.n_rows = r;
        o.n_cols = c;
        o.ld = r > 1 ? r : 1;
        o.dtype = dtype_of<eT>::value;
        o.flags = KIND;
        o.gen[0] = g0;
        o.gen[1] = g1;
        return o;
    }
    int flatten(Flat& f) const { return f.leaf(operand(), nullptr); }
};

template <class eT>
using GenEye = Gen<eT, COOT_OPERAND_GEN_EYE>;
template <class eT>
using GenFill = Gen<eT, COOT_OPERAND_GEN_FILL>;
template <class eT>
using GenLin = Gen<eT, COOT_OPERAND_GEN_LINSPACE>;

// --------------------------------------------------------- evaluation core
namespace detail {

inline coot_operand make_operand(const void* p, int64_t r, int64_t c, int64_t ld, int dt, uint32_t flags = 0)
{
    coot_operand o;
    std::memset(&o, 0, sizeof o);
    o.ptr = const_cast<void*>(p);
    o.n_rows = r;
    o.n_cols = c;
    o.ld = ld;
    o.dtype = dt;
    o.flags = flags;
    return o;
}

template <class T1>
int eval_into(const T1& X, const coot_operand& out)
{
    Flat f;
    X.flatten(f);
    const coot_expr e = f.expr();
    return coot_eval(&e, f.ops.data(), (int)f.ops.size(), &out, get_stream());
}

// host-result reduction of a tree
template <class R, class T1>
R reduce_host(int red_op, const T1& X, int out_dt)
{
    Flat f;
    X.flatten(f);
    const coot_expr e = f.expr();
    R r{};
    coot_operand out = make_operand(&r, 1, 1, 1, out_dt, COOT_OPERAND_HOST);
    check(coot_reduce(red_op, -1, &e, f.ops.data(), (int)f.ops.size(), &out, get_stream()));
    return r;
}

}  // namespace detail

// ------------------------------------------------------------------- Mat
template <class eT>
class Mat : public Base<eT, Mat<eT>> {
    static_assert(std::is_same<eT, float>::value || std::is_same<eT, double>::value ||
                      std::is_same<eT, int32_t>::value || std::is_same<eT, uint32_t>::value,
                  "Mat<eT>: eT is float, double, int32_t or uint32_t");

public:
    Mat() = default;
    Mat(int64_t r, int64_t c) { set_size(r, c); }
    // non-owning: wrap caller-owned device memory (e.g. a torch tensor)
    Mat(eT* dev, int64_t r, int64_t c, int64_t ld = 0) : mem_(dev), r_(r), c_(c), ld_(ld ? ld : (r > 1 ? r : 1)) {}
    Mat(const Mat& o) { *this = o; }
    Mat(Mat&& o) noexcept { swap(o); }
    template <class T1>
    Mat(const Base<eT, T1>& X)
    {
        *this = X;
    }
    ~Mat() { release(); }

    // a matrix that wraps caller memory keeps it: the value is copied in
    Mat& operator=(Mat&& o)
    {
        if (this == &o) return *this;
        if (mem_ && !owns_) {
            assign(o);
        } else {
            release();
            swap(o);
        }
        return *this;
    }
    Mat& operator=(const Mat& o)
    {
        if (this != &o) assign(o);
        return *this;
    }
    template <class T1>
    Mat& operator=(const Base<eT, T1>& X)
    {
        assign(X.get_ref());
        return *this;
    }

    // compound assignment: the operand is read in place (no temporary)
    template <class T1>
    Mat& operator+=(const Base<eT, T1>& X) { return *this = eGlue<Mat, T1, COOT_PLUS>(*this, X.get_ref()); }
    template <class T1>
    Mat& operator-=(const Base<eT, T1>& X) { return *this = eGlue<Mat, T1, COOT_MINUS>(*this, X.get_ref()); }
    template <class T1>
    Mat& operator%=(const Base<eT, T1>& X) { return *this = eGlue<Mat, T1, COOT_SCHUR>(*this, X.get_ref()); }
    template <class T1>
    Mat& operator/=(const Base<eT, T1>& X) { return *this = eGlue<Mat, T1, COOT_DIV>(*this, X.get_ref()); }
    Mat& operator+=(double k) { return *this = eOp<Mat, COOT_SCAL_PLUS>(*this, k); }
    Mat& operator-=(double k) { return *this = eOp<Mat, COOT_SCAL_MINUS_POST>(*this, k); }
    Mat& operator*=(double k) { return *this = eOp<Mat, COOT_SCAL_TIMES>(*this, k); }
    Mat& operator/=(double k) { return *this = eOp<Mat, COOT_SCAL_DIV_POST>(*this, k); }

    // shape and memory
    int64_t n_rows() const { return r_; }
    int64_t n_cols() const { return c_; }
    int64_t n_elem() const { return r_ * c_; }
    int64_t ld() const { return ld_; }
    bool is_empty() const { return r_ * c_ == 0; }
    bool is_square() const { return r_ == c_; }
    bool is_vec() const { return r_ == 1 || c_ == 1; }
    eT* memptr() { return mem_; }
    const eT* memptr() const { return mem_; }
    coot_operand operand() const { return detail::make_operand(mem_, r_, c_, ld_, dtype_of<eT>::value); }
    int flatten(Flat& f) const { return f.leaf(operand(), this); }

    void set_size(int64_t r, int64_t c)
    {
        if (r == r_ && c == c_) return;
        if (mem_ && !owns_) throw std::runtime_error("coot: cannot resize a matrix that wraps external memory");
        release();
        if (r < 0 || c < 0) throw std::runtime_error("coot: negative size");
        if (r * c > 0)
            check_hip(hipMallocAsync((void**)&mem_, (size_t)(r * c) * sizeof(eT), get_stream()), "hipMallocAsync");
        owns_ = mem_ != nullptr;
        r_ = r;
        c_ = c;
        ld_ = r > 1 ? r : 1;
    }
    void reset() { set_size(0, 0); }

    // Table 1 generators as members
    Mat& fill(double k) { return *this = GenFill<eT>(r_, c_, k); }
    Mat& ones() { return fill(1.0); }
    Mat& zeros() { return fill(0.0); }
    Mat& eye() { return *this = GenEye<eT>(r_, c_); }
    Mat& ones(int64_t r, int64_t c) { set_size(r, c); return ones(); }
    Mat& zeros(int64_t r, int64_t c) { set_size(r, c); return zeros(); }
    Mat& eye(int64_t r, int64_t c) { set_size(r, c); return eye(); }

    // Table 1 submatrix views
    subview<eT> submat(int64_t p, int64_t q, int64_t r, int64_t s) const;
    subview<eT> rows(int64_t a, int64_t b) const { return submat(a, 0, b, c_ - 1); }
    subview<eT> cols(int64_t c, int64_t d) const { return submat(0, c, r_ - 1, d); }
    subview<eT> row(int64_t i) const { return rows(i, i); }
    subview<eT> col(int64_t j) const { return cols(j, j); }
    subview<eT> diag(int64_t k = 0) const;

    Op<Mat, op_htrans> t() const { return Op<Mat, op_htrans>(*this); }

    // host transfers (synchronous), column-major host arrays of n_rows x n_cols
    void copy_from_host(const eT* h)
    {
        if (n_elem() == 0) return;
        check_hip(hipMemcpy2DAsync(mem_, (size_t)ld_ * sizeof(eT), h, (size_t)(r_ > 0 ? r_ : 1) * sizeof(eT),
                                   (size_t)r_ * sizeof(eT), (size_t)c_, hipMemcpyHostToDevice, get_stream()),
                  "hipMemcpy2DAsync");
        check_hip(hipStreamSynchronize(get_stream()), "hipStreamSynchronize");
    }
    void copy_to_host(eT* h) const
    {
        if (n_elem() == 0) return;
        check_hip(hipMemcpy2DAsync(h, (size_t)(r_ > 0 ? r_ : 1) * sizeof(eT), mem_, (size_t)ld_ * sizeof(eT),
                                   (size_t)r_ * sizeof(eT), (size_t)c_, hipMemcpyDeviceToHost, get_stream()),
                  "hipMemcpy2DAsync");
        check_hip(hipStreamSynchronize(get_stream()), "hipStreamSynchronize");
    }

private:
    eT* mem_ = nullptr;
    int64_t r_ = 0, c_ = 0, ld_ = 1;
    bool owns_ = false;

    void release()
    {
        if (owns_ && mem_) (void)hipFreeAsync(mem_, get_stream());
        mem_ = nullptr;
        owns_ = false;
        r_ = c_ = 0;
        ld_ = 1;
    }
    void swap(Mat& o) noexcept
    {
        std::swap(mem_, o.mem_);
        std::swap(r_, o.r_);
        std::swap(c_, o.c_);
        std::swap(ld_, o.ld_);
        std::swap(owns_, o.owns_);
    }
    // Delayed evaluation: the whole expression becomes one coot_eval.  When
    // the destination must change shape, or the library refuses to write in
    // place (an operand read transposed is the destination), the value goes
    // to a fresh matrix that then replaces this one.
    template <class T1>
    void assign(const T1& X)
    {
        const int64_t r = X.n_rows(), c = X.n_cols();
        if (r == r_ && c == c_) {
            const int rc = detail::eval_into(X, operand());
            if (rc != COOT_ERR_ALIAS) {
                check(rc);
                return;
            }
            if (mem_ && !owns_) {
                Mat tmp(r, c);
                check(detail::eval_into(X, tmp.operand()));
                check(detail::eval_into(tmp, operand()));
                return;
            }
        } else if (mem_ && !owns_) {
            throw std::runtime_error("coot: cannot resize a matrix that wraps external memory");
        }
        Mat tmp(r, c);
        check(detail::eval_into(X, tmp.operand()));
        release();
        swap(tmp);
    }
    friend class subview<eT>;
};

template <class eT>
struct is_leaf<Mat<eT>> : std::true_type {};

// Col and Row: matrices with one column / one row
template <class eT>
class Col : public Mat<eT> {
public:
    Col() = default;
    explicit Col(int64_t n) : Mat<eT>(n, 1) {}
    Col(eT* dev, int64_t n) : Mat<eT>(dev, n, 1) {}
    template <class T1>
    Col(const Base<eT, T1>& X) : Mat<eT>(X)
    {
    }
    template <class T1>
    Col& operator=(const Base<eT, T1>& X)
    {
        Mat<eT>::operator=(X);
        return *this;
    }
};

template <class eT>
class Row : public Mat<eT> {
public:
    Row() = default;
    explicit Row(int64_t n) : Mat<eT>(1, n) {}
    Row(eT* dev, int64_t n) : Mat<eT>(dev, 1, n, 1) {}
    template <class T1>
    Row(const Base<eT, T1>& X) : Mat<eT>(X)
    {
    }
    template <class T1>
    Row& operator=(const Base<eT, T1>& X)
    {
        Mat<eT>::operator=(X);
        return *this;
    }
};

using fmat = Mat<float>;
using mat = Mat<double>;
using dmat = Mat<double>;
using fvec = Col<float>;
using vec = Col<double>;
using fcolvec = Col<float>;
using colvec = Col<double>;
using frowvec = Row<float>;
using rowvec = Row<double>;
// 32-bit integer matrices: values widen exactly to FP64 for the arithmetic;
// storing into them drops the fraction toward zero and clamps to the range
using imat = Mat<int32_t>;
using umat = Mat<uint32_t>;
using ivec = Col<int32_t>;
using uvec = Col<uint32_t>;
using irowvec = Row<int32_t>;
using urowvec = Row<uint32_t>;

// --------------------------------------------------------------- subview
// A view into a matrix: a strided operand (ptr, shape, ld) that is both a leaf
// of expressions and a destination.
template <class eT>
class subview : public Base<eT, subview<eT>> {
public:
    subview(const eT* p, int64_t r, int64_t c, int64_t ld) : p_(const_cast<eT*>(p)), r_(r), c_(c), ld_(ld) {}
    subview(const subview&) = default;
    int64_t n_rows() const { return r_; }
    int64_t n_cols() const { return c_; }
    int64_t n_elem() const { return r_ * c_; }
    coot_operand operand() const { return detail::make_operand(p_, r_, c_, ld_, dtype_of<eT>::value); }
    int flatten(Flat& f) const { return f.leaf(operand(), p_); }

    template <class T1>
    subview& operator=(const Base<eT, T1>& X)
    {
        const T1& E = X.get_ref();
        if (E.n_rows() != r_ || E.n_cols() != c_) throw std::runtime_error("coot: view and expression shapes differ");
        const int rc = detail::eval_into(E, operand());
        if (rc == COOT_ERR_ALIAS) {
            Mat<eT> tmp(r_, c_);
            check(detail::eval_into(E, tmp.operand()));
            check(detail::eval_into(tmp, operand()));
            return *this;
        }
        check(rc);
        return *this;
    }
    subview& operator=(const subview& o) { return operator=<subview>(o); }
    subview& fill(double k) { return *this = GenFill<eT>(r_, c_, k); }
    template <class T1>
    subview& operator+=(const Base<eT, T1>& X) { return *this = eGlue<subview, T1, COOT_PLUS>(*this, X.get_ref()); }
    template <class T1>
    subview& operator-=(const Base<eT, T1>& X) { return *this = eGlue<subview, T1, COOT_MINUS>(*this, X.get_ref()); }
    template <class T1>
    subview& operator%=(const Base<eT, T1>& X) { return *this = eGlue<subview, T1, COOT_SCHUR>(*this, X.get_ref()); }
    subview& operator+=(double k) { return *this = eOp<subview, COOT_SCAL_PLUS>(*this, k); }
    subview& operator-=(double k) { return *this = eOp<subview, COOT_SCAL_MINUS_POST>(*this, k); }
    subview& operator*=(double k) { return *this = eOp<subview, COOT_SCAL_TIMES>(*this, k); }
    subview& operator/=(double k) { return *this = eOp<subview, COOT_SCAL_DIV_POST>(*this, k); }

private:
    eT* p_;
    int64_t r_, c_, ld_;
};

template <class eT>
subview<eT> Mat<eT>::submat(int64_t p, int64_t q, int64_t r, int64_t s) const
{
    if (p < 0 || q < 0 || r >= r_ || s >= c_ || r + 1 < p || s + 1 < q)
        throw std::runtime_error("coot: submat bounds outside the matrix");
    return subview<eT>(mem_ + p + q * ld_, r - p + 1, s - q + 1, ld_);
}

// .diag(k): a 1 x n operand whose ld is the parent's + 1
template <class eT>
subview<eT> Mat<eT>::diag(int64_t k) const
{
    const int64_t r0 = k < 0 ? -k : 0, c0 = k > 0 ? k : 0;
    int64_t n = r_ - r0 < c_ - c0 ? r_ - r0 : c_ - c0;
    if (n < 0) n = 0;
    return subview<eT>(mem_ + r0 + c0 * ld_, 1, n, ld_ + 1);
}

// ------------------------------------------------------------ generators
// eye<fmat>(r, c), ones<fmat>(r, c), zeros<fmat>(r, c), linspace<fvec>(a, b, n)
template <class M>
GenEye<typename M::elem_type> eye(int64_t r, int64_t c)
{
    return GenEye<typename M::elem_type>(r, c);
}
template <class M>
GenFill<typename M::elem_type> ones(int64_t r, int64_t c)
{
    return GenFill<typename M::elem_type>(r, c, 1.0);
}
template <class M>
GenFill<typename M::elem_type> zeros(int64_t r, int64_t c)
{
    return GenFill<typename M::elem_type>(r, c, 0.0);
}
template <class V>
GenLin<typename V::elem_type> linspace(double start, double end, int64_t n)
{
    constexpr bool row = std::is_base_of<Row<typename V::elem_type>, V>::value;
    return GenLin<typename V::elem_type>(row ? 1 : n, row ? n : 1, start, end);
}

// ------------------------------------------------- transpose and rewrites
template <class eT, class T1>
Op<T1, op_htrans> trans(const Base<eT, T1>& X)
{
    return Op<T1, op_htrans>(X.get_ref());
}
// exact simplifications chosen while the type is built (Section 7):
// trans(trans(X)) = X; generators are their own transposes (shape swapped)
template <class T1>
const T1& trans(const Op<T1, op_htrans>& X)
{
    return X.m;
}
template <class eT>
GenEye<eT> trans(const GenEye<eT>& X)
{
    return GenEye<eT>(X.c, X.r);
}
template <class eT>
GenFill<eT> trans(const GenFill<eT>& X)
{
    return GenFill<eT>(X.c, X.r, X.g0);
}
template <class eT>
GenLin<eT> trans(const GenLin<eT>& X)
{
    return GenLin<eT>(X.c, X.r, X.g0, X.g1);
}

// conversion: conv_to<fmat>::from(expr) (fused into the kernel, Section 7)
template <class M>
struct conv_to {
    template <class eT, class T1>
    static mtOp<typename M::elem_type, T1> from(const Base<eT, T1>& X)
    {
        return mtOp<typename M::elem_type, T1>(X.get_ref());
    }
};

// ------------------------------------------------------ element-wise ops
// scalar overloads take part only for arithmetic scalars (else A + B would
// match the scalar form exactly and never reach the element-wise one)
template <class S>
using if_arith = std::enable_if_t<std::is_arithmetic<S>::value, int>;

#define COOT_GLUE(OPER, CODE)                                                                   \
    template <class eT, class T1, class T2>                                                     \
    eGlue<T1, T2, CODE> OPER(const Base<eT, T1>& a, const Base<eT, T2>& b)                      \
    {                                                                                           \
        return eGlue<T1, T2, CODE>(a.get_ref(), b.get_ref());                                   \
    }
COOT_GLUE(operator+, COOT_PLUS)
COOT_GLUE(operator-, COOT_MINUS)
COOT_GLUE(operator%, COOT_SCHUR)
COOT_GLUE(operator/, COOT_DIV)
COOT_GLUE(operator>, COOT_GT)
COOT_GLUE(operator<, COOT_LT)
COOT_GLUE(operator>=, COOT_GE)
COOT_GLUE(operator<=, COOT_LE)
COOT_GLUE(operator==, COOT_EQ)
COOT_GLUE(operator!=, COOT_NE)
#undef COOT_GLUE

// A * B between two matrices is a matrix product, not an element-wise
// operation: not part of this library (use % for the element-wise product).
template <class eT, class T1, class T2>
void operator*(const Base<eT, T1>&, const Base<eT, T2>&) = delete;

// scalar forms: X op k and k op X
#define COOT_SCALAR(OPER, POST, PRE)                                                            \
    template <class eT, class T1, class S, if_arith<S> = 0>                                     \
    eOp<T1, POST> OPER(const Base<eT, T1>& a, S k)                                              \
    {                                                                                           \
        return eOp<T1, POST>(a.get_ref(), (double)k);                                           \
    }                                                                                           \
    template <class eT, class T1, class S, if_arith<S> = 0>                                     \
    eOp<T1, PRE> OPER(S k, const Base<eT, T1>& a)                                               \
    {                                                                                           \
        return eOp<T1, PRE>(a.get_ref(), (double)k);                                            \
    }
// a + k = k + a and a * k = k * a exactly; k - a, k / a, k > a have forms of their own
COOT_SCALAR(operator+, COOT_SCAL_PLUS, COOT_SCAL_PLUS)
COOT_SCALAR(operator-, COOT_SCAL_MINUS_POST, COOT_SCAL_MINUS_PRE)
COOT_SCALAR(operator*, COOT_SCAL_TIMES, COOT_SCAL_TIMES)
COOT_SCALAR(operator/, COOT_SCAL_DIV_POST, COOT_SCAL_DIV_PRE)
COOT_SCALAR(operator>, COOT_SCAL_GT, COOT_SCAL_LT)
COOT_SCALAR(operator<, COOT_SCAL_LT, COOT_SCAL_GT)
COOT_SCALAR(operator>=, COOT_SCAL_GE, COOT_SCAL_LE)
COOT_SCALAR(operator<=, COOT_SCAL_LE, COOT_SCAL_GE)
COOT_SCALAR(operator==, COOT_SCAL_EQ, COOT_SCAL_EQ)
COOT_SCALAR(operator!=, COOT_SCAL_NE, COOT_SCAL_NE)
#undef COOT_SCALAR

// -X = X * (-1), exact
template <class eT, class T1>
eOp<T1, COOT_SCAL_TIMES> operator-(const Base<eT, T1>& a)
{
    return eOp<T1, COOT_SCAL_TIMES>(a.get_ref(), -1.0);
}

#define COOT_UNARY(NAME, CODE)                                                                  \
    template <class eT, class T1>                                                               \
    eOp<T1, CODE> NAME(const Base<eT, T1>& a)                                                   \
    {                                                                                           \
        return eOp<T1, CODE>(a.get_ref());                                                      \
    }
COOT_UNARY(exp, COOT_EXP)
COOT_UNARY(log, COOT_LOG)
COOT_UNARY(sqrt, COOT_SQRT)
COOT_UNARY(abs, COOT_ABS)
COOT_UNARY(log10, COOT_LOG10)
COOT_UNARY(log2, COOT_LOG2)
COOT_UNARY(exp2, COOT_EXP2)
COOT_UNARY(square, COOT_SQUARE)
COOT_UNARY(floor, COOT_FLOOR)
COOT_UNARY(ceil, COOT_CEIL)
COOT_UNARY(round, COOT_ROUND)
COOT_UNARY(trunc, COOT_TRUNC)
COOT_UNARY(sign, COOT_SIGN)
COOT_UNARY(cos, COOT_COS)
COOT_UNARY(sin, COOT_SIN)
COOT_UNARY(tan, COOT_TAN)
COOT_UNARY(acos, COOT_ACOS)
COOT_UNARY(asin, COOT_ASIN)
COOT_UNARY(atan, COOT_ATAN)
COOT_UNARY(cosh, COOT_COSH)
COOT_UNARY(sinh, COOT_SINH)
COOT_UNARY(tanh, COOT_TANH)
#undef COOT_UNARY

template <class eT, class T1, class S, if_arith<S> = 0>
eOp<T1, COOT_SCAL_POW> pow(const Base<eT, T1>& a, S k)
{
    return eOp<T1, COOT_SCAL_POW>(a.get_ref(), (double)k);
}

// ------------------------------------------------ scalar-valued functions
template <class eT, class T1>
red_t<eT> accu(const Base<eT, T1>& X)
{
    return detail::reduce_host<red_t<eT>>(COOT_RED_ACCU, X.get_ref(), dtype_of<red_t<eT>>::value);
}
template <class eT, class T1, class T2>
red_t<eT> dot(const Base<eT, T1>& A, const Base<eT, T2>& B)
{
    return detail::reduce_host<red_t<eT>>(COOT_RED_DOT, eGlue<T1, T2, COOT_SCHUR>(A.get_ref(), B.get_ref()),
                                          dtype_of<red_t<eT>>::value);
}
// norm(X, p): p = 1 or 2, or "inf", "-inf", "fro" (Table 5)
template <class eT, class T1>
red_t<eT> norm(const Base<eT, T1>& X, int p = 2)
{
    if (p != 1 && p != 2) throw std::runtime_error("coot: norm(X, p) takes p = 1 or 2");
    return detail::reduce_host<red_t<eT>>(p == 1 ? COOT_RED_NORM1 : COOT_RED_NORM2, X.get_ref(),
                                          dtype_of<red_t<eT>>::value);
}
template <class eT, class T1>
red_t<eT> norm(const Base<eT, T1>& X, const char* p)
{
    const std::string s(p);
    const int op = s == "inf" ? COOT_RED_NORMINF
                              : (s == "-inf" ? COOT_RED_NORMNEGINF : (s == "fro" ? COOT_RED_NORM2 : -1));
    if (op < 0) throw std::runtime_error("coot: norm(X, p) takes \"inf\", \"-inf\" or \"fro\"");
    return detail::reduce_host<red_t<eT>>(op, X.get_ref(), dtype_of<red_t<eT>>::value);
}
template <class eT, class T1>
red_t<eT> min(const Base<eT, T1>& X)
{
    return detail::reduce_host<red_t<eT>>(COOT_RED_MIN, X.get_ref(), dtype_of<red_t<eT>>::value);
}
template <class eT, class T1>
red_t<eT> max(const Base<eT, T1>& X)
{
    return detail::reduce_host<red_t<eT>>(COOT_RED_MAX, X.get_ref(), dtype_of<red_t<eT>>::value);
}
template <class eT, class T1>
uword index_min(const Base<eT, T1>& X)
{
    return detail::reduce_host<uword>(COOT_RED_INDEX_MIN, X.get_ref(), COOT_U64);
}
template <class eT, class T1>
uword index_max(const Base<eT, T1>& X)
{
    return detail::reduce_host<uword>(COOT_RED_INDEX_MAX, X.get_ref(), COOT_U64);
}
template <class eT, class T1>
bool all(const Base<eT, T1>& X)
{
    return detail::reduce_host<uword>(COOT_RED_ALL, X.get_ref(), COOT_U64) != 0;
}
template <class eT, class T1>
bool any(const Base<eT, T1>& X)
{
    return detail::reduce_host<uword>(COOT_RED_ANY, X.get_ref(), COOT_U64) != 0;
}
// statistics over all elements (the vector forms of Table 6)
template <class eT, class T1>
red_t<eT> mean(const Base<eT, T1>& X)
{
    return detail::reduce_host<red_t<eT>>(COOT_RED_MEAN, X.get_ref(), dtype_of<red_t<eT>>::value);
}
template <class eT, class T1>
red_t<eT> var(const Base<eT, T1>& X)
{
    return detail::reduce_host<red_t<eT>>(COOT_RED_VAR, X.get_ref(), dtype_of<red_t<eT>>::value);
}
template <class eT, class T1>
red_t<eT> stddev(const Base<eT, T1>& X)
{
    return detail::reduce_host<red_t<eT>>(COOT_RED_STDDEV, X.get_ref(), dtype_of<red_t<eT>>::value);
}
// trace(A): the sum of the leading diagonal
template <class eT>
red_t<eT> trace(const Mat<eT>& A)
{
    return accu(A.diag());
}

// ------------------------------------------------ vector-valued functions
// sum / min / max / mean / var / stddev along dim (0: per column -> 1 x n_cols,
// 1: per row -> n_rows x 1), Table 6; the result is a new matrix
namespace detail {
template <class eT, class T1>
Mat<red_t<eT>> reduce_dim(int red_op, const T1& X, int dim)
{
    if (dim != 0 && dim != 1) throw std::runtime_error("coot: dim is 0 or 1");
    Mat<red_t<eT>> out(dim == 0 ? 1 : X.n_rows(), dim == 0 ? X.n_cols() : 1);
    Flat f;
    X.flatten(f);
    const coot_expr e = f.expr();
    coot_operand o = out.operand();
    if (dim == 0) o.ld = 1;
    check(coot_reduce(red_op, dim, &e, f.ops.data(), (int)f.ops.size(), &o, get_stream()));
    return out;
}
}  // namespace detail

#define COOT_DIMRED(NAME, CODE)                                                                 \
    template <class eT, class T1>                                                               \
    Mat<red_t<eT>> NAME(const Base<eT, T1>& X, int dim)                                         \
    {                                                                                           \
        return detail::reduce_dim<eT>(CODE, X.get_ref(), dim);                                  \
    }
COOT_DIMRED(sum, COOT_RED_SUM)
COOT_DIMRED(min, COOT_RED_MIN)
COOT_DIMRED(max, COOT_RED_MAX)
COOT_DIMRED(mean, COOT_RED_MEAN)
COOT_DIMRED(var, COOT_RED_VAR)
COOT_DIMRED(stddev, COOT_RED_STDDEV)
#undef COOT_DIMRED

// diagvec(A, k): the k-th diagonal as a column (Table 6)
template <class eT>
Op<subview<eT>, op_htrans> diagvec(const Mat<eT>& A, int64_t k = 0)
{
    return Op<subview<eT>, op_htrans>(A.diag(k));
}

// ---------------------------------------------------------- introspection
// The node array and operand table an expression flattens to (host only; no
// device work).  Used to check the expression types against the ABI.
template <class eT, class T1>
Flat describe(const Base<eT, T1>& X)
{
    Flat f;
    X.get_ref().flatten(f);
    return f;
}

}  // namespace coot

#endif  // COOT_HPP
