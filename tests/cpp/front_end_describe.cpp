// Host-only check of the C++ front end (include/coot.hpp): prints, one JSON
// line per expression, the postfix node array and operand table the
// expression type flattens to, for comparison with the trees the Python
// binding builds for the same expressions.  Device pointers are stand-ins
// (nothing is dereferenced and no device call is made).
#include <cstdio>
#include <type_traits>

#include "coot.hpp"

using namespace coot;

template <class eT, class T1>
static void show(const char* name, const Base<eT, T1>& X)
{
    const Flat f = describe(X);
    std::printf("{\"name\": \"%s\", \"nodes\": [", name);
    for (size_t i = 0; i < f.nodes.size(); ++i)
        std::printf("%s[%d, %d, %d, %.17g]", i ? ", " : "", f.nodes[i].op, f.nodes[i].a, f.nodes[i].b, f.nodes[i].k);
    std::printf("], \"ops\": [");
    for (size_t i = 0; i < f.ops.size(); ++i)
        std::printf("%s[%lld, %lld, %lld, %d, %u, %.17g, %.17g, %lld]", i ? ", " : "", (long long)f.ops[i].n_rows,
                    (long long)f.ops[i].n_cols, (long long)f.ops[i].ld, f.ops[i].dtype, f.ops[i].flags, f.ops[i].gen[0],
                    f.ops[i].gen[1], (long long)((const char*)f.ops[i].ptr - (const char*)nullptr));
    std::printf("]}\n");
}

int main()
{
    float* P = reinterpret_cast<float*>(uintptr_t(1) << 40);
    double* Q = reinterpret_cast<double*>(uintptr_t(1) << 41);
    fmat A(P, 30, 20), B(P + 1000, 30, 20), C(P + 2000, 30, 20), D(P + 3000, 30, 20), T(P + 4000, 20, 30);
    mat X(Q, 30, 20);
    int32_t* I = reinterpret_cast<int32_t*>(uintptr_t(1) << 42);
    imat K(I, 30, 20), L(I + 1000, 30, 20);
    // exact rewrites chosen by overload resolution while the type is built
    static_assert(std::is_same<decltype(trans(trans(A))), const fmat&>::value, "trans(trans(A)) is A");
    static_assert(std::is_same<decltype(trans(eye<fmat>(3, 4))), GenEye<float>>::value, "trans(eye) is eye");
    static_assert(std::is_same<decltype(A + B), eGlue<fmat, fmat, COOT_PLUS>>::value, "A + B is an eGlue");
    static_assert(std::is_same<decltype(2.0 * A), eOp<fmat, COOT_SCAL_TIMES>>::value, "k * A is an eOp");

    show("small_Y", 2.5 * A + B % C - exp(D));
    show("accu_AB", A % B);
    show("trans_sum", trans(T) + 0.5 * B);
    show("double_trans", trans(trans(A)) % A);
    show("scalars", 1.0 - A / 2.0 + (3.0 / B) - (A - 4.0));
    show("relational", (A > 0.3) % (0.3 > B) + (A <= B) - (A != 2.0));
    show("funcs", sqrt(abs(A)) % log(abs(B) + 1.0) + pow(abs(C), 1.5) - tanh(D));
    show("conv", conv_to<fmat>::from(X * 2.0) + A);
    show("neg", -A + B);
    show("eye_fill", A + 3.0 * eye<fmat>(30, 20) - ones<fmat>(30, 20) + trans(eye<fmat>(20, 30)));
    show("linspace", linspace<fvec>(-1.0, 2.0, 30) * 2.0);
    show("views", A.submat(1, 2, 10, 12) + B.submat(0, 0, 9, 10));
    show("diag", trans(A.diag(3)));
    show("integers", conv_to<fmat>::from(K * 2 + L / 3) + A);
    show("integer_conv", conv_to<imat>::from(A * 1000.0) + K);
    return 0;
}
