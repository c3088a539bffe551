// Conjugate gradients on A = D[free, free] (validation solve): CSR SpMV with
// one thread per row, dot products reduced in a fixed two-level order, FP64
// vectors and residuals whatever the precision of the matrix values.
#include "nla_internal.hpp"
#include <cmath>
#include <mutex>
#include <vector>

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <class T>
__global__ void k_spmv(int n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci, const T *__restrict__ v,
                       const double *__restrict__ x, double *__restrict__ y)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t t = rp[i]; t < rp[i + 1]; t++) s += (double)v[t] * x[ci[t]];
    y[i] = s;
}

// r = b - y, p = r
__global__ void k_resid(int n, const double *__restrict__ b, const double *__restrict__ y, double *__restrict__ r,
                        double *__restrict__ p)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = b[i] - y[i];
    r[i] = v;
    p[i] = v;
}

// per-block partial sums of x.y, block tree in fixed order
__global__ __launch_bounds__(256) void k_dot_part(int n, const double *__restrict__ x, const double *__restrict__ y,
                                                  double *__restrict__ part)
{
    __shared__ double sh[256];
    int i = blockIdx.x * 256 + threadIdx.x;
    sh[threadIdx.x] = i < n ? x[i] * y[i] : 0.0;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_dot_final(int nb, const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// u += alpha p ; r -= alpha Ap
__global__ void k_update(int n, double alpha, const double *__restrict__ p, const double *__restrict__ Ap,
                         double *__restrict__ u, double *__restrict__ r)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u[i] += alpha * p[i];
    r[i] -= alpha * Ap[i];
}

// p = r + beta p
__global__ void k_dir(int n, double beta, const double *__restrict__ r, double *__restrict__ p)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    p[i] = r[i] + beta * p[i];
}

struct CgScratch {
    std::vector<void *> ptrs;
    ~CgScratch()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    int get(double **p, size_t n)
    {
        if (hipMalloc((void **)p, sizeof(double) * (n ? n : 1)) != hipSuccess) {
            nla_set_error("hipMalloc failed in CG");
            return NLA_E_NOMEM;
        }
        ptrs.push_back(*p);
        return NLA_OK;
    }
};

static int dot(int n, const double *x, const double *y, double *part, double *out, double *host, hipStream_t s)
{
    const int nb = (int)grid_for(n, 256);
    k_dot_part<<<nb, 256, 0, s>>>(n, x, y, part);
    k_dot_final<<<1, 256, 0, s>>>(nb, part, out);
    NLA_HIP(hipMemcpyAsync(host, out, sizeof(double), hipMemcpyDeviceToHost, s));
    NLA_HIP(hipStreamSynchronize(s));
    return NLA_OK;
}

// The iteration on caller-provided scratch: r, p, Ap [n], part [ceil(n/256)],
// out [1]; every value is written before it is read.
static int cg_solve(const nla_plan *P, const double *b, double *u, double rtol, int32_t maxit, int32_t *iters,
                    double *relres, hipStream_t s, double *r, double *p, double *Ap, double *part, double *out)
{
    const int n = P->n_free;
    const unsigned g = grid_for(n, 256);
    auto spmv = [&](const double *x, double *y) {
        if (P->val_dtype == NLA_DTYPE_F64)
            k_spmv<double><<<g, 256, 0, s>>>(n, P->a_rowptr, P->a_col, (const double *)P->a_val, x, y);
        else
            k_spmv<float><<<g, 256, 0, s>>>(n, P->a_rowptr, P->a_col, (const float *)P->a_val, x, y);
    };
    double bb = 0.0, rr = 0.0, pAp = 0.0;
    NLA_TRY(dot(n, b, b, part, out, &bb, s));
    const double nb = std::sqrt(bb);
    spmv(u, Ap);
    k_resid<<<g, 256, 0, s>>>(n, b, Ap, r, p);
    NLA_TRY(dot(n, r, r, part, out, &rr, s));
    int it = 0;
    while (std::sqrt(rr) > rtol * nb && it < maxit) {
        spmv(p, Ap);
        NLA_TRY(dot(n, p, Ap, part, out, &pAp, s));
        if (!(pAp > 0.0)) {
            nla_set_error("CG breakdown: p.Ap = %g", pAp);
            return NLA_E_NOT_CONVERGED;
        }
        double alpha = rr / pAp;
        k_update<<<g, 256, 0, s>>>(n, alpha, p, Ap, u, r);
        double rr_new = 0.0;
        NLA_TRY(dot(n, r, r, part, out, &rr_new, s));
        k_dir<<<g, 256, 0, s>>>(n, rr_new / rr, r, p);
        rr = rr_new;
        it++;
    }
    NLA_HIP(hipGetLastError());
    NLA_HIP(hipStreamSynchronize(s));
    *iters = it;
    *relres = nb > 0 ? std::sqrt(rr) / nb : 0.0;
    if (std::sqrt(rr) > rtol * nb) {
        nla_set_error("CG did not reach rtol %g in %d iterations (relres %g)", rtol, it, *relres);
        return NLA_E_NOT_CONVERGED;
    }
    return NLA_OK;
}

int nla_cg_run(const nla_plan *P, const double *b, double *u, double rtol, int32_t maxit, int32_t *iters,
               double *relres, hipStream_t s)
{
    const int n = P->n_free;
    *iters = 0;
    *relres = 0.0;
    if (n == 0) return NLA_OK;
    CgScratch S;
    double *r, *p, *Ap, *part, *out;
    NLA_TRY(S.get(&r, n));
    NLA_TRY(S.get(&p, n));
    NLA_TRY(S.get(&Ap, n));
    NLA_TRY(S.get(&part, grid_for(n, 256)));
    NLA_TRY(S.get(&out, 1));
    return cg_solve(P, b, u, rtol, maxit, iters, relres, s, r, p, Ap, part, out);
}

// ---------------------------------------------------------------------------
// Allocation-free CG.  Its scratch (r, p, Ap for up to NLA_CG_NOALLOC_MAX_FREE
// free nodes, the dot products' block sums and their result) is a file-scope
// device array: each device the library runs on holds its own copy, 24 MiB and
// 32 KiB, from the module's load until the process ends.  Host code never
// passes the array's name to a kernel: the name is a host-side stand-in, and
// the copy's device address comes from hipGetSymbolAddress, taken once per
// device with that device current and kept in cg_scratch_ptr.
namespace {
constexpr size_t CG_PART_MAX = (NLA_CG_NOALLOC_MAX_FREE + 255) / 256;
constexpr size_t CG_SCRATCH_DOUBLES = 3 * (size_t)NLA_CG_NOALLOC_MAX_FREE + CG_PART_MAX + 32;
constexpr int CG_MAX_DEVICES = 64;
std::mutex cg_scratch_mu;
double *cg_scratch_ptr[CG_MAX_DEVICES] = {};
} // namespace

static __device__ __align__(256) double scratch[CG_SCRATCH_DOUBLES];

// the device address of `scratch` on device dev (the current device)
static int cg_scratch_on(int dev, double **out)
{
    std::lock_guard<std::mutex> lock(cg_scratch_mu);
    if (dev < 0 || dev >= CG_MAX_DEVICES) {
        nla_set_error("device %d is beyond the %d devices the allocation-free CG serves", dev, CG_MAX_DEVICES);
        return NLA_E_DEVICE;
    }
    if (!cg_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            nla_set_error("hipGetSymbolAddress of the CG scratch failed on device %d: %s", dev, hipGetErrorString(e));
            return NLA_E_DEVICE;
        }
        cg_scratch_ptr[dev] = (double *)ptr;
    }
    *out = cg_scratch_ptr[dev];
    return NLA_OK;
}

extern "C" int nla_cg_noalloc(const nla_plan *P, const double *b, double *u, double rtol, int32_t maxit,
                              int32_t *iters, double *relres, void *stream)
{
    if (!P || !b || !u || !iters || !relres) { nla_set_error("null argument"); return NLA_E_INVALID; }
    if (!P->assembled) { nla_set_error("nla_assemble has not run"); return NLA_E_STATE; }
    if (maxit < 1 || !(rtol > 0)) { nla_set_error("maxit >= 1 and rtol > 0 required"); return NLA_E_INVALID; }
    const int n = P->n_free;
    if (n > NLA_CG_NOALLOC_MAX_FREE) {
        nla_set_error("%d free nodes exceed the allocation-free CG's scratch (at most %d); use nla_cg", n,
                      NLA_CG_NOALLOC_MAX_FREE);
        return NLA_E_INVALID;
    }
    int dev = -1;
    NLA_HIP(hipGetDevice(&dev));
    if (dev != P->device) {
        nla_set_error("the plan lives on device %d but device %d is current", P->device, dev);
        return NLA_E_DEVICE;
    }
    *iters = 0;
    *relres = 0.0;
    if (n == 0) return NLA_OK;
    double *base = nullptr;
    NLA_TRY(cg_scratch_on(dev, &base));
    double *r = base, *p = r + NLA_CG_NOALLOC_MAX_FREE, *Ap = p + NLA_CG_NOALLOC_MAX_FREE;
    double *part = Ap + NLA_CG_NOALLOC_MAX_FREE, *out = part + CG_PART_MAX;
    return cg_solve(P, b, u, rtol, maxit, iters, relres, (hipStream_t)stream, r, p, Ap, part, out);
}
