// elementwise.hip -- the arithmetic layer applied elementwise, so that each
// DD/QD operation can be compared bit for bit with an independent host
// implementation of the same published algorithm.
#include "internal.hpp"
#include "mp.hpp"

namespace hcn {

template <class R>
__global__ void k_elementwise(int op, int count, const double *__restrict__ a,
                              const double *__restrict__ b, double *__restrict__ out) {
    constexpr int P = limbs<R>::P;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    switch (op) {
        case 0: case 1: case 2: case 3: {
            R x, y;
            rload(a + (size_t)q * P, x);
            rload(b + (size_t)q * P, y);
            R z = op == 0 ? add(x, y) : op == 1 ? sub(x, y) : op == 2 ? mul(x, y) : div(x, y);
            rstore(out + (size_t)q * P, z);
            break;
        }
        case 4: {
            R x;
            rload(a + (size_t)q * P, x);
            rstore(out + (size_t)q * P, sqrt(x));
            break;
        }
        case 5: {
            R x;
            rload(a + (size_t)q * P, x);
            rstore(out + (size_t)q * P, mul_d(x, b[q]));
            break;
        }
        case 10: case 11: case 12: case 13: {
            const cx<R> x = cload<R>(a + (size_t)q * 2 * P);
            const cx<R> y = cload<R>(b + (size_t)q * 2 * P);
            const cx<R> z = op == 10 ? cadd(x, y) : op == 11 ? csub(x, y)
                          : op == 12 ? cmul(x, y) : cmul_conj(x, y);
            cstore(out + (size_t)q * 2 * P, z);
            break;
        }
        case 14:
            rstore(out + (size_t)q * P, cnorm2(cload<R>(a + (size_t)q * 2 * P)));
            break;
        case 15: {
            R s;
            rload(b + (size_t)q * P, s);
            cstore(out + (size_t)q * 2 * P, cscale(s, cload<R>(a + (size_t)q * 2 * P)));
            break;
        }
        case 20: {
            double s, e;
            eft_sum(a[q], b[q], s, e);
            out[2 * q] = s;
            out[2 * q + 1] = e;
            break;
        }
        case 21: {
            double s, e;
            eft_fast_sum(a[q], b[q], s, e);
            out[2 * q] = s;
            out[2 * q + 1] = e;
            break;
        }
        case 22: {
            double p, e;
            eft_prod(a[q], b[q], p, e);
            out[2 * q] = p;
            out[2 * q + 1] = e;
            break;
        }
        default:
            break;
    }
}

int launch_elementwise(int op, int P, int count, const double *a, const double *b, double *out,
                       hipStream_t stream) {
    if (count == 0) return 0;
    dim3 grid((count + 255) / 256);
    if (P == 1)
        hipLaunchKernelGGL(k_elementwise<double>, grid, dim3(256), 0, stream, op, count, a, b, out);
    else if (P == 2)
        hipLaunchKernelGGL(k_elementwise<dd>, grid, dim3(256), 0, stream, op, count, a, b, out);
    else
        hipLaunchKernelGGL(k_elementwise<qd>, grid, dim3(256), 0, stream, op, count, a, b, out);
    return (int)hipGetLastError();
}

}  // namespace hcn
