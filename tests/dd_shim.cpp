// Host build of the device double-double arithmetic (csrc/dd.hpp), for the
// CPU pins of its error bounds (tests/test_dd_pins.py).  Compiled for the
// host only; every operation is IEEE binary64 with explicit fma and no other
// contraction, so it computes the same bits as the device.
#include "dd.hpp"

extern "C" void dds_op(int op, const double* a, const double* b, const double* c, const double* d,
                       double* out) {
    const dd A = mk_dd(a[0], a[1]), B = mk_dd(b[0], b[1]), C = mk_dd(c[0], c[1]),
             D = mk_dd(d[0], d[1]);
    dd r = mk_dd(0.0, 0.0);
    switch (op) {
        case 0: r = add(A, B); break;
        case 1: r = add_acc(A, B); break;
        case 2: r = sub(A, B); break;
        case 3: r = mul(A, B); break;
        case 4: r = mul(A, B.hi); break;
        case 5: r = div(A, B); break;
        case 6: r = mul_add(A, B, C); break;
        case 7: r = mul_sub(A, B, C, D); break;
        case 8: r = two_sum(A.hi, B.hi); break;
        case 9: r = two_prod(A.hi, B.hi); break;
        case 10: r = fast_two_sum(A.hi, B.hi); break;
        default: break;
    }
    out[0] = r.hi;
    out[1] = r.lo;
}
