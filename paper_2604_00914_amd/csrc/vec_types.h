// 16-byte vector element types for the sparse x dense-block kernels.
//
// Every dense row is processed in 16-byte pieces: 2 doubles, 4 floats, 1 complex
// double or 2 complex floats.  The traits give the per-piece multiply-add with a
// matrix value and the real-scalar epilogue.  All arithmetic is written as
// explicit fused multiply-adds in a fixed order (the library is built with
// -ffp-contract=off), so a column's result does not depend on which kernel
// variant or batch position computed it.
#pragma once

#include <hip/hip_runtime.h>

namespace afsi {

struct TrR64 {
    using vec = double2;
    using val = double;
    using scal = double;
    static constexpr int E = 2;  // elements per vector
    __device__ static inline vec zero() { return make_double2(0.0, 0.0); }
    __device__ static inline val val_zero() { return 0.0; }
    __device__ static inline vec fma_val(val a, vec w, vec acc) {
        acc.x = __builtin_fma(a, w.x, acc.x);
        acc.y = __builtin_fma(a, w.y, acc.y);
        return acc;
    }
    __device__ static inline vec scale(scal s, vec a) { return make_double2(s * a.x, s * a.y); }
    __device__ static inline vec axpy(scal s, vec x, vec y) {
        return make_double2(__builtin_fma(s, x.x, y.x), __builtin_fma(s, x.y, y.y));
    }
    __device__ static inline vec sub(vec a, vec b) { return make_double2(a.x - b.x, a.y - b.y); }
};

struct TrR32 {
    using vec = float4;
    using val = float;
    using scal = float;
    static constexpr int E = 4;
    __device__ static inline vec zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ static inline val val_zero() { return 0.f; }
    __device__ static inline vec fma_val(val a, vec w, vec acc) {
        acc.x = __builtin_fmaf(a, w.x, acc.x);
        acc.y = __builtin_fmaf(a, w.y, acc.y);
        acc.z = __builtin_fmaf(a, w.z, acc.z);
        acc.w = __builtin_fmaf(a, w.w, acc.w);
        return acc;
    }
    __device__ static inline vec scale(scal s, vec a) {
        return make_float4(s * a.x, s * a.y, s * a.z, s * a.w);
    }
    __device__ static inline vec axpy(scal s, vec x, vec y) {
        return make_float4(__builtin_fmaf(s, x.x, y.x), __builtin_fmaf(s, x.y, y.y),
                           __builtin_fmaf(s, x.z, y.z), __builtin_fmaf(s, x.w, y.w));
    }
    __device__ static inline vec sub(vec a, vec b) {
        return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
    }
};

// One complex double per vector: (x, y) = (re, im).
struct TrC128 {
    using vec = double2;
    using val = double2;
    using scal = double;
    static constexpr int E = 1;
    __device__ static inline vec zero() { return make_double2(0.0, 0.0); }
    __device__ static inline val val_zero() { return make_double2(0.0, 0.0); }
    __device__ static inline vec fma_val(val a, vec w, vec acc) {
        acc.x = __builtin_fma(a.x, w.x, acc.x);
        acc.x = __builtin_fma(-a.y, w.y, acc.x);
        acc.y = __builtin_fma(a.x, w.y, acc.y);
        acc.y = __builtin_fma(a.y, w.x, acc.y);
        return acc;
    }
    __device__ static inline vec scale(scal s, vec a) { return TrR64::scale(s, a); }
    __device__ static inline vec axpy(scal s, vec x, vec y) { return TrR64::axpy(s, x, y); }
    __device__ static inline vec sub(vec a, vec b) { return TrR64::sub(a, b); }
};

// Two complex floats per vector: (x, y) and (z, w).
struct TrC64 {
    using vec = float4;
    using val = float2;
    using scal = float;
    static constexpr int E = 2;
    __device__ static inline vec zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ static inline val val_zero() { return make_float2(0.f, 0.f); }
    __device__ static inline vec fma_val(val a, vec w, vec acc) {
        acc.x = __builtin_fmaf(a.x, w.x, acc.x);
        acc.x = __builtin_fmaf(-a.y, w.y, acc.x);
        acc.y = __builtin_fmaf(a.x, w.y, acc.y);
        acc.y = __builtin_fmaf(a.y, w.x, acc.y);
        acc.z = __builtin_fmaf(a.x, w.z, acc.z);
        acc.z = __builtin_fmaf(-a.y, w.w, acc.z);
        acc.w = __builtin_fmaf(a.x, w.w, acc.w);
        acc.w = __builtin_fmaf(a.y, w.z, acc.w);
        return acc;
    }
    __device__ static inline vec scale(scal s, vec a) { return TrR32::scale(s, a); }
    __device__ static inline vec axpy(scal s, vec x, vec y) { return TrR32::axpy(s, x, y); }
    __device__ static inline vec sub(vec a, vec b) { return TrR32::sub(a, b); }
};

// Single-element traits for blocks whose rows are not 16-byte aligned.  The
// multiply-add and epilogue sequences match the vector traits element by element.
struct SR64 {
    using vec = double;
    using val = double;
    using scal = double;
    __device__ static inline vec zero() { return 0.0; }
    __device__ static inline val val_zero() { return 0.0; }
    __device__ static inline vec fma_val(val a, vec w, vec acc) { return __builtin_fma(a, w, acc); }
    __device__ static inline vec scale(scal s, vec a) { return s * a; }
    __device__ static inline vec axpy(scal s, vec x, vec y) { return __builtin_fma(s, x, y); }
    __device__ static inline vec sub(vec a, vec b) { return a - b; }
};
struct SR32 {
    using vec = float;
    using val = float;
    using scal = float;
    __device__ static inline vec zero() { return 0.f; }
    __device__ static inline val val_zero() { return 0.f; }
    __device__ static inline vec fma_val(val a, vec w, vec acc) { return __builtin_fmaf(a, w, acc); }
    __device__ static inline vec scale(scal s, vec a) { return s * a; }
    __device__ static inline vec axpy(scal s, vec x, vec y) { return __builtin_fmaf(s, x, y); }
    __device__ static inline vec sub(vec a, vec b) { return a - b; }
};
using SC128 = TrC128;
struct SC64 {
    using vec = float2;
    using val = float2;
    using scal = float;
    __device__ static inline vec zero() { return make_float2(0.f, 0.f); }
    __device__ static inline val val_zero() { return make_float2(0.f, 0.f); }
    __device__ static inline vec fma_val(val a, vec w, vec acc) {
        acc.x = __builtin_fmaf(a.x, w.x, acc.x);
        acc.x = __builtin_fmaf(-a.y, w.y, acc.x);
        acc.y = __builtin_fmaf(a.x, w.y, acc.y);
        acc.y = __builtin_fmaf(a.y, w.x, acc.y);
        return acc;
    }
    __device__ static inline vec scale(scal s, vec a) { return make_float2(s * a.x, s * a.y); }
    __device__ static inline vec axpy(scal s, vec x, vec y) {
        return make_float2(__builtin_fmaf(s, x.x, y.x), __builtin_fmaf(s, x.y, y.y));
    }
    __device__ static inline vec sub(vec a, vec b) { return make_float2(a.x - b.x, a.y - b.y); }
};

// Streaming (non-temporal) accesses for blocks read or written once per product,
// so that they do not evict the gathered source rows from L2 and the MALL.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
__device__ inline double nt_load(const double *p) { return __builtin_nontemporal_load(p); }
__device__ inline float nt_load(const float *p) { return __builtin_nontemporal_load(p); }
__device__ inline double2 nt_load(const double2 *p) {
    const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(p));
    return make_double2(v.x, v.y);
}
__device__ inline float4 nt_load(const float4 *p) {
    const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline float2 nt_load(const float2 *p) {
    const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2 *>(p));
    return make_float2(v.x, v.y);
}
__device__ inline void nt_store(double v, double *p) { __builtin_nontemporal_store(v, p); }
__device__ inline void nt_store(float v, float *p) { __builtin_nontemporal_store(v, p); }
__device__ inline void nt_store(double2 v, double2 *p) {
    const nt_d2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_d2 *>(p));
}
__device__ inline void nt_store(float4 v, float4 *p) {
    const nt_f4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_f4 *>(p));
}
__device__ inline void nt_store(float2 v, float2 *p) {
    const nt_f2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_f2 *>(p));
}

// Epilogue shared by every variant:  r = sigma*acc;  r = tau*w + r;  r = r - v;  r = alpha*x + r
template <class Tr>
__device__ inline typename Tr::vec clenshaw_combine(typename Tr::scal sigma, typename Tr::scal tau,
                                                    typename Tr::vec acc, typename Tr::vec w) {
    return Tr::axpy(tau, w, Tr::scale(sigma, acc));
}

}  // namespace afsi
