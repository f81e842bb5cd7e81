// C ABI of the slab 3D real FFT: plans, argument checks and pass sequencing.
// Every argument is validated on the host before the first HIP call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/gfft.h"
#include "kernels.h"

struct gfft_plan {
    int64_t n, x, p, y, batch, k;
    int64_t rs;  // reals between real rows: n, or n + 2 in place
    int lg_n, lg_x, lg_y, lg_p;
    gfft_dtype dtype;
    uint32_t flags;
    int device;
    void* tw;  // W_N^m, m = 0..N-1, in the working precision
    // z rows per grid: X * N (slab), X * Y (pencil: x and y extents local)
    int64_t zrows;
    // pencil plans: pr x pc process grid, this rank's column `col`, its kz
    // width w = N/(2 pc) (+1 for the last column); g = pc/pr y-pencil blocks
    // per second-exchange peer (pr <= pc), or h = pr/pc peers per y-pencil
    // block (pr > pc, the block then packed into h runs of N/pr rows)
    bool pencil;
    int64_t pr, pc, col, w, g, h;
    int lg_w0, lg_g, lg_h;
};

namespace {

constexpr uint32_t kKnownFlags =
    GFFT_FUSE_PACK | GFFT_MFMA_BF16X2 | GFFT_MFMA_BF16X3 | GFFT_INPLACE | GFFT_PACK_PAPER_ORDER;

int ilog2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}
bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// exp(-2 pi i m / n) for a power of two n >= 4: reduce to a quadrant and to
// an angle of at most pi/4 in exact integer arithmetic, evaluate in long
// double, round once to double.
void unit_root(int64_t m, int64_t n, double* re, double* im) {
    const int64_t q4 = n / 4;
    const int64_t quad = (m / q4) & 3;
    const int64_t r = m % q4;  // angle 2 pi r / n in [0, pi/2)
    long double c, s;
    const long double two_pi = 6.283185307179586476925286766559005768L;
    if (2 * r <= q4) {
        const long double a = two_pi * (long double)r / (long double)n;
        c = cosl(a);
        s = sinl(a);
    } else {  // pi/2 - a' with a' <= pi/4
        const long double a = two_pi * (long double)(q4 - r) / (long double)n;
        c = sinl(a);
        s = cosl(a);
    }
    long double cr, ci;  // (c + i s) * i^quad = exp(+i theta)
    switch (quad) {
        case 0: cr = c; ci = s; break;
        case 1: cr = -s; ci = c; break;
        case 2: cr = -c; ci = -s; break;
        default: cr = s; ci = -c; break;
    }
    *re = (double)cr;
    *im = -(double)ci;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

gfft_status check_ptr(const void* p) {
    if (!p) return GFFT_E_INVALID_ARG;
    if (!aligned16(p)) return GFFT_E_ALIGN;
    return GFFT_OK;
}

bool overlap(const void* a, int64_t na, const void* b, int64_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + uint64_t(nb) && y < x + uint64_t(na);
}

int64_t real_size(const gfft_plan* p) { return p->batch * p->zrows * p->rs; }
int64_t cplx_count(const gfft_plan* p) { return p->batch * p->zrows * p->k; }
int64_t elt(const gfft_plan* p) { return p->dtype == GFFT_F64 ? 8 : 4; }
int64_t real_bytes(const gfft_plan* p) { return real_size(p) * elt(p); }
int64_t cplx_bytes(const gfft_plan* p) { return cplx_count(p) * 2 * elt(p); }

bool paper(const gfft_plan* p) { return (p->flags & GFFT_PACK_PAPER_ORDER) != 0; }

// Rows of the half spectrum that the z passes write or read: natural, or one
// of the two send orders when the pack is fused.
gfft::row_map zmap(const gfft_plan* p) {
    if (p->pencil) {
        gfft::row_map m{p->lg_n, p->lg_x, p->lg_n, p->rs, 0};
        m.pencil = 1;
        m.lg_rows = p->lg_x + p->lg_y;
        m.lg_w = p->lg_w0;
        m.pc_last = int(p->pc - 1);
        return m;
    }
    const bool packed = (p->flags & GFFT_FUSE_PACK) != 0;
    return gfft::row_map{p->lg_n, p->lg_x, packed ? p->lg_y : p->lg_n, p->rs,
                         packed && paper(p) ? 1 : 0};
}

// The send order of the standalone pack.
gfft::row_map packmap(const gfft_plan* p) {
    return gfft::row_map{p->lg_n, p->lg_x, p->lg_y, p->rs, paper(p) ? 1 : 0};
}

// y lines of a [batch][X][N][K] half spectrum: natural, send order
// [p][X][N/p][K], or the paper's order [N][X][K] (slab transposed).
gfft::line_map ymap(const gfft_plan* p) {
    gfft::line_map lm;
    if (p->pencil) {  // [batch][pc][X][Y][w]: y = c' Y + y_l, planes x_l
        lm.b_hi = p->pc * p->x * p->y * p->w;
        lm.lg_bx = p->lg_x;
        lm.b_lo = p->y * p->w;
        lm.s_hi = p->x * p->y * p->w;
        lm.s_lo = p->w;
        lm.lg_y = p->lg_y;
        return lm;
    }
    const bool packed = (p->flags & GFFT_FUSE_PACK) != 0;
    lm.b_hi = p->x * p->n * p->k;
    lm.lg_bx = p->lg_x;
    if (packed && paper(p)) {
        lm.b_lo = p->k;
        lm.s_hi = 0;
        lm.s_lo = p->x * p->k;
        lm.lg_y = p->lg_n;
        return lm;
    }
    const int64_t yy = packed ? p->y : p->n;
    lm.b_lo = yy * p->k;
    lm.s_hi = p->x * yy * p->k;
    lm.s_lo = p->k;
    lm.lg_y = packed ? p->lg_y : p->lg_n;
    return lm;
}

// x lines of a received pencil: [batch][N][Y][K] (x = i X + x_l slowest), or
// in the paper's chunk order [batch][p][Y][X][K] with the chunk transpose of
// step 4 folded into the addressing (a batch of Y line sets, K columns each).
gfft::line_map xmap(const gfft_plan* p) {
    gfft::line_map lm;
    if (p->pencil && p->h > 1) {  // [batch][pr][X][N/pr][w] = [batch][N][N/pr][w]
        lm.b_hi = p->n * (p->n / p->pr) * p->w;
        lm.b_lo = 0;
        lm.s_hi = 0;
        lm.s_lo = (p->n / p->pr) * p->w;
        lm.lg_bx = 0;
        lm.lg_y = p->lg_n;
        return lm;
    }
    if (p->pencil) {  // [batch][pr][g][X][Y][w]: x = r X + x_l, line sets (item, g_l)
        lm.b_hi = p->pc * p->x * p->y * p->w;
        lm.lg_bx = p->lg_g;
        lm.b_lo = p->x * p->y * p->w;
        lm.s_hi = p->g * p->x * p->y * p->w;
        lm.s_lo = p->y * p->w;
        lm.lg_y = p->lg_x;
        return lm;
    }
    if (paper(p)) {
        lm.b_hi = p->n * p->y * p->k;
        lm.b_lo = p->x * p->k;
        lm.lg_bx = p->lg_y;
        lm.s_hi = p->y * p->x * p->k;
        lm.s_lo = p->k;
        lm.lg_y = p->lg_x;
        return lm;
    }
    lm.b_hi = p->n * p->y * p->k;
    lm.b_lo = 0;
    lm.s_hi = 0;
    lm.s_lo = p->y * p->k;
    lm.lg_bx = 0;
    lm.lg_y = p->lg_n;
    return lm;
}

gfft_status hip_status(hipError_t e) { return e == hipSuccess ? GFFT_OK : GFFT_E_HIP; }

// The plan's tables live on the device that was current at creation, and
// its kernels must run there: exec calls refuse any other current device
// (checked last, after the arguments).
gfft_status check_device(const gfft_plan* p) {
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess) return GFFT_E_HIP;
    return d == p->device ? GFFT_OK : GFFT_E_INVALID_ARG;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

bool f64(const gfft_plan* p) { return p->dtype == GFFT_F64; }

gfft_status run_z_r2c(const gfft_plan* p, const void* in, void* out, double scale,
                      bool weighted, hipStream_t s) {
    const double me = scale, mi = weighted ? 2.0 * scale : scale;
    return hip_status(gfft::launch_z_r2c(f64(p), int(p->n), in, out, p->tw,
                                         p->batch * p->zrows, zmap(p), me, mi, s));
}

gfft_status run_z_c2r(const gfft_plan* p, const void* in, void* out, double scale,
                      bool weighted, hipStream_t s) {
    const double me = scale, mi = weighted ? 0.5 * scale : scale;
    return hip_status(gfft::launch_z_c2r(f64(p), int(p->n), in, out, p->tw,
                                         p->batch * p->zrows, zmap(p), me, mi, s));
}

int mfma_terms(const gfft_plan* p) {
    if (p->flags & GFFT_MFMA_BF16X3) return 3;
    if (p->flags & GFFT_MFMA_BF16X2) return 2;
    return 0;
}

// copy: the pass's loads and stores without its transform (gfft_exec_pass_copy)
gfft_status run_y(const gfft_plan* p, void* data, int sign, hipStream_t s, bool copy = false) {
    const int64_t cols = p->pencil ? p->w : p->k;
    return hip_status(gfft::launch_strided(f64(p), int(p->n), 0, copy ? -1 : mfma_terms(p), sign,
                                           data, p->tw, cols, p->batch * p->x, ymap(p), s));
}

gfft_status run_x(const gfft_plan* p, void* data, int sign, hipStream_t s, bool copy = false) {
    int64_t cols = paper(p) ? p->k : p->y * p->k;
    int64_t sets = paper(p) ? p->batch * p->y : p->batch;
    if (p->pencil) {
        cols = p->h > 1 ? (p->n / p->pr) * p->w : p->y * p->w;
        sets = p->h > 1 ? p->batch : p->batch * p->g;
    }
    return hip_status(gfft::launch_strided(f64(p), int(p->n), 1, copy ? -1 : mfma_terms(p), sign,
                                           data, p->tw, cols, sets, xmap(p), s));
}

// `real` and `cplx` are the two buffers of a z pass: distinct and disjoint,
// or the very same buffer for an in-place plan.
gfft_status check_r2c_args(const gfft_plan* p, const void* real, const void* cplx) {
    if (!p) return GFFT_E_INVALID_ARG;
    gfft_status st = check_ptr(real);
    if (st != GFFT_OK) return st;
    if ((st = check_ptr(cplx)) != GFFT_OK) return st;
    if (p->flags & GFFT_INPLACE) return real == cplx ? GFFT_OK : GFFT_E_INVALID_ARG;
    if (overlap(real, real_bytes(p), cplx, cplx_bytes(p))) return GFFT_E_INVALID_ARG;
    return GFFT_OK;
}

// Step 1 or its inverse as one pass per plane where a plane fits on a CU
// and that is measured faster (FP32, N = 64..256; not for pencil plans,
// whose z output is cut into kz chunks, nor with the matrix-core stage,
// which belongs to the y pass).
bool plane_pass(const gfft_plan* p, bool fwd) {
    return !p->pencil && mfma_terms(p) == 0 && gfft::plane_supported(f64(p), int(p->n), fwd);
}

gfft_status run_plane(const gfft_plan* p, bool fwd, const void* in, void* out, double scale,
                      bool weighted, hipStream_t s) {
    const double me = scale, mi = weighted ? (fwd ? 2.0 : 0.5) * scale : scale;
    return hip_status(gfft::launch_plane(f64(p), fwd, int(p->n), in, out, p->tw,
                                         p->batch * p->x, zmap(p), me, mi, s));
}

gfft_status forward(const gfft_plan* p, const void* in, void* out, double scale,
                    bool weighted, void* stream) {
    gfft_status st = check_r2c_args(p, in, out);
    if (st != GFFT_OK) return st;
    if (p->pencil) return GFFT_E_UNSUPPORTED;
    if (!std::isfinite(scale)) return GFFT_E_INVALID_ARG;
    if ((st = check_device(p)) != GFFT_OK) return st;
    hipStream_t s = as_stream(stream);
    if (plane_pass(p, true)) {
        if ((st = run_plane(p, true, in, out, scale, weighted, s)) != GFFT_OK) return st;
    } else {
        if ((st = run_z_r2c(p, in, out, scale, weighted, s)) != GFFT_OK) return st;
        if ((st = run_y(p, out, -1, s)) != GFFT_OK) return st;
    }
    if (p->p == 1) st = run_x(p, out, -1, s);
    return st;
}

gfft_status inverse(const gfft_plan* p, void* in, void* out, double scale, bool weighted,
                    void* stream) {
    gfft_status st = check_r2c_args(p, out, in);
    if (st != GFFT_OK) return st;
    if (p->pencil) return GFFT_E_UNSUPPORTED;
    if (!std::isfinite(scale)) return GFFT_E_INVALID_ARG;
    if ((st = check_device(p)) != GFFT_OK) return st;
    hipStream_t s = as_stream(stream);
    if (p->p == 1 && (st = run_x(p, in, +1, s)) != GFFT_OK) return st;
    if (plane_pass(p, false)) return run_plane(p, false, in, out, scale, weighted, s);
    if ((st = run_y(p, in, +1, s)) != GFFT_OK) return st;
    return run_z_c2r(p, in, out, scale, weighted, s);
}

// Second-exchange pack of a pencil plan with pr > pc: every y-pencil block
// [X][Y][w] (per grid and c') splits into h = pr/pc runs [X][N/pr][w], run s
// for peer c' h + s -- the slab pack's permutation with Y rows in h chunks.
gfft_status pencil_pack(const gfft_plan* p, const void* src, void* dst, bool to_send,
                        void* stream) {
    if (p->h == 1) return GFFT_E_UNSUPPORTED;  // blocks already contiguous
    gfft_status st = check_ptr(src);
    if (st != GFFT_OK || (st = check_ptr(dst)) != GFFT_OK) return st;
    const int64_t bytes = p->batch * p->pc * p->x * p->y * p->w * 2 * elt(p);
    if (overlap(src, bytes, dst, bytes)) return GFFT_E_INVALID_ARG;
    if ((st = check_device(p)) != GFFT_OK) return st;
    return hip_status(gfft::launch_pack(f64(p), src, dst, p->batch * p->pc * p->h * p->x,
                                        p->lg_x, p->lg_h, p->y, p->y / p->h, p->w, to_send,
                                        as_stream(stream)));
}

// The current device, if it is a gfx950.
gfft_status usable_device(int* dev) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return GFFT_E_NO_DEVICE;
    if (hipGetDevice(dev) != hipSuccess) return GFFT_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, *dev) != hipSuccess) return GFFT_E_HIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return GFFT_E_NO_DEVICE;
    return GFFT_OK;
}

// FP64 twiddles W_N^m, m = 0..N-1, rounded once to the working precision,
// into a device table owned by the plan.
gfft_status upload_twiddles(gfft_plan* p) {
    const int64_t n = p->n;
    const size_t bytes = size_t(n) * 2 * (p->dtype == GFFT_F64 ? 8 : 4);
    std::vector<unsigned char> host(bytes);
    for (int64_t m = 0; m < n; ++m) {
        double re, im;
        unit_root(m, n, &re, &im);
        if (p->dtype == GFFT_F64) {
            double* h = reinterpret_cast<double*>(host.data());
            h[2 * m] = re;
            h[2 * m + 1] = im;
        } else {
            float* h = reinterpret_cast<float*>(host.data());
            h[2 * m] = float(re);
            h[2 * m + 1] = float(im);
        }
    }
    if (hipMalloc(&p->tw, bytes) != hipSuccess) {
        p->tw = nullptr;
        return GFFT_E_NOMEM;
    }
    if (hipMemcpy(p->tw, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p->tw);
        p->tw = nullptr;
        return GFFT_E_HIP;
    }
    return GFFT_OK;
}

}  // namespace

extern "C" {

int gfft_version(void) { return 100; }

const char* gfft_status_string(gfft_status st) {
    switch (st) {
        case GFFT_OK: return "success";
        case GFFT_E_INVALID_ARG: return "invalid argument";
        case GFFT_E_UNSUPPORTED: return "unsupported size or flag combination";
        case GFFT_E_ALIGN: return "data pointer not 16-byte aligned";
        case GFFT_E_NOMEM: return "out of device memory for plan tables";
        case GFFT_E_HIP: return "HIP runtime or kernel launch failure";
        case GFFT_E_NO_DEVICE: return "no usable gfx950 device";
        case GFFT_STATUS_MAX_ENUM: break;
    }
    return "unknown status";
}

gfft_status gfft_plan_create(gfft_plan** out, int64_t n, gfft_dtype dtype, int64_t slab_x,
                             int64_t batch, uint32_t flags) {
    if (!out) return GFFT_E_INVALID_ARG;
    *out = nullptr;
    if (dtype != GFFT_F64 && dtype != GFFT_F32) return GFFT_E_INVALID_ARG;
    if (flags & ~kKnownFlags) return GFFT_E_INVALID_ARG;
    if (batch < 1 || slab_x < 1 || n < 1) return GFFT_E_INVALID_ARG;
    if (!pow2(n) || n < 16 || n > 4096) return GFFT_E_UNSUPPORTED;
    if (slab_x > n || n % slab_x != 0) return GFFT_E_INVALID_ARG;
    const uint32_t mf = flags & (GFFT_MFMA_BF16X2 | GFFT_MFMA_BF16X3);
    if (mf == (GFFT_MFMA_BF16X2 | GFFT_MFMA_BF16X3)) return GFFT_E_INVALID_ARG;
    if (mf && (dtype != GFFT_F32 || n < 32)) return GFFT_E_UNSUPPORTED;
    if ((flags & GFFT_INPLACE) && (flags & GFFT_FUSE_PACK)) return GFFT_E_UNSUPPORTED;
    if ((flags & GFFT_PACK_PAPER_ORDER) && slab_x == n) return GFFT_E_UNSUPPORTED;
    // sizes must stay addressable with 64-bit element offsets
    const int64_t k = n / 2 + 1;
    if (batch > (int64_t(1) << 62) / (slab_x * n * k * 2 * 8)) return GFFT_E_UNSUPPORTED;

    int dev = 0;
    gfft_status st = usable_device(&dev);
    if (st != GFFT_OK) return st;

    gfft_plan* p = new (std::nothrow) gfft_plan;
    if (!p) return GFFT_E_NOMEM;
    p->n = n;
    p->x = slab_x;
    p->p = n / slab_x;
    p->y = n / p->p;
    p->batch = batch;
    p->k = k;
    p->rs = (flags & GFFT_INPLACE) ? n + 2 : n;
    p->lg_n = ilog2(n);
    p->lg_x = ilog2(slab_x);
    p->lg_p = ilog2(p->p);
    p->lg_y = ilog2(p->y);
    p->dtype = dtype;
    p->flags = flags;
    p->device = dev;
    p->tw = nullptr;
    p->zrows = slab_x * n;
    p->pencil = false;
    p->pr = p->p;
    p->pc = 1;
    p->col = 0;
    p->w = k;
    p->g = 1;
    p->h = 1;
    p->lg_w0 = 0;
    p->lg_g = 0;
    p->lg_h = 0;
    if ((st = upload_twiddles(p)) != GFFT_OK) {
        delete p;
        return st;
    }
    *out = p;
    return GFFT_OK;
}

gfft_status gfft_pencil_plan_create(gfft_plan** out, int64_t n, gfft_dtype dtype,
                                    int64_t grid_r, int64_t grid_c, int64_t col,
                                    int64_t batch, uint32_t flags) {
    if (!out) return GFFT_E_INVALID_ARG;
    *out = nullptr;
    if (dtype != GFFT_F64 && dtype != GFFT_F32) return GFFT_E_INVALID_ARG;
    if (flags & ~kKnownFlags) return GFFT_E_INVALID_ARG;
    if (batch < 1 || n < 1 || grid_r < 1 || grid_c < 1) return GFFT_E_INVALID_ARG;
    if (col < 0 || col >= grid_c) return GFFT_E_INVALID_ARG;
    if (!pow2(n) || n < 16 || n > 4096) return GFFT_E_UNSUPPORTED;
    if (!pow2(grid_r) || !pow2(grid_c)) return GFFT_E_INVALID_ARG;
    // kz is cut into grid_c chunks of N/(2 grid_c) bins; x into grid_r slabs
    if (grid_c > n / 2 || grid_r > n) return GFFT_E_UNSUPPORTED;
    const uint32_t mf = flags & (GFFT_MFMA_BF16X2 | GFFT_MFMA_BF16X3);
    if (mf == (GFFT_MFMA_BF16X2 | GFFT_MFMA_BF16X3)) return GFFT_E_INVALID_ARG;
    if (mf && (dtype != GFFT_F32 || n < 32)) return GFFT_E_UNSUPPORTED;
    if (flags & (GFFT_FUSE_PACK | GFFT_INPLACE | GFFT_PACK_PAPER_ORDER)) return GFFT_E_UNSUPPORTED;
    const int64_t k = n / 2 + 1, xr = n / grid_r, yc = n / grid_c;
    const int64_t w = n / (2 * grid_c) + (col == grid_c - 1 ? 1 : 0);
    // every buffer (real rows, first-exchange order, y/x pencil) must stay
    // addressable with 64-bit byte offsets
    int64_t item = xr * yc * n * 8;
    if (xr * yc * k * 16 > item) item = xr * yc * k * 16;
    if (grid_c * xr * yc * w * 16 > item) item = grid_c * xr * yc * w * 16;
    if (batch > (int64_t(1) << 62) / item) return GFFT_E_UNSUPPORTED;

    int dev = 0;
    gfft_status st = usable_device(&dev);
    if (st != GFFT_OK) return st;
    gfft_plan* p = new (std::nothrow) gfft_plan;
    if (!p) return GFFT_E_NOMEM;
    p->n = n;
    p->x = xr;
    p->y = yc;
    p->p = grid_r * grid_c;
    p->batch = batch;
    p->k = k;
    p->rs = n;
    p->lg_n = ilog2(n);
    p->lg_x = ilog2(xr);
    p->lg_y = ilog2(yc);
    p->lg_p = ilog2(p->p);
    p->dtype = dtype;
    p->flags = flags;
    p->device = dev;
    p->tw = nullptr;
    p->zrows = xr * yc;
    p->pencil = true;
    p->pr = grid_r;
    p->pc = grid_c;
    p->col = col;
    p->w = w;
    p->g = grid_r <= grid_c ? grid_c / grid_r : 1;
    p->h = grid_r > grid_c ? grid_r / grid_c : 1;
    p->lg_w0 = ilog2(n / (2 * grid_c));
    p->lg_g = ilog2(p->g);
    p->lg_h = ilog2(p->h);
    if ((st = upload_twiddles(p)) != GFFT_OK) {
        delete p;
        return st;
    }
    *out = p;
    return GFFT_OK;
}

gfft_status gfft_plan_destroy(gfft_plan* p) {
    if (!p) return GFFT_OK;
    gfft_status st = GFFT_OK;
    if (p->tw && hipFree(p->tw) != hipSuccess) st = GFFT_E_HIP;
    delete p;
    return st;
}

gfft_status gfft_plan_query(const gfft_plan* p, gfft_plan_sizes* s) {
    if (!p || !s) return GFFT_E_INVALID_ARG;
    s->n = p->n;
    s->slab_x = p->x;
    s->ranks = p->p;
    s->batch = p->batch;
    s->k = p->k;
    s->real_bytes = real_bytes(p);
    s->complex_bytes = cplx_bytes(p);
    if (p->pencil) {
        s->pencil_bytes = p->batch * p->pc * p->x * p->y * p->w * 2 * elt(p);
        s->chunk_bytes = p->x * p->y * p->w * 2 * elt(p);
    } else {
        s->pencil_bytes = p->batch * p->n * p->y * p->k * 2 * elt(p);
        s->chunk_bytes = p->x * p->y * p->k * 2 * elt(p);
    }
    s->grid_r = p->pr;
    s->grid_c = p->pc;
    s->col = p->col;
    s->y_local = p->pencil ? p->y : p->n;
    s->kz_width = p->w;
    return GFFT_OK;
}

gfft_status gfft_exec_r2c(const gfft_plan* p, const void* in, void* out, void* stream) {
    return forward(p, in, out, 1.0, false, stream);
}

gfft_status gfft_exec_c2r_adjoint(const gfft_plan* p, const void* in, void* out,
                                  double scale, void* stream) {
    return forward(p, in, out, scale, true, stream);
}

gfft_status gfft_exec_c2r(const gfft_plan* p, void* in, void* out, double scale,
                          void* stream) {
    return inverse(p, in, out, scale, false, stream);
}

gfft_status gfft_exec_r2c_adjoint(const gfft_plan* p, void* in, void* out, double scale,
                                  void* stream) {
    return inverse(p, in, out, scale, true, stream);
}

gfft_status gfft_pack_slab_for_alltoall(const gfft_plan* p, const void* src, void* dst,
                                        void* stream) {
    if (!p) return GFFT_E_INVALID_ARG;
    if (p->pencil) return pencil_pack(p, src, dst, true, stream);
    gfft_status st = check_ptr(src);
    if (st != GFFT_OK || (st = check_ptr(dst)) != GFFT_OK) return st;
    if (overlap(src, cplx_bytes(p), dst, cplx_bytes(p))) return GFFT_E_INVALID_ARG;
    if ((st = check_device(p)) != GFFT_OK) return st;
    if (paper(p))
        return hip_status(gfft::launch_pack_rows(f64(p), src, dst, p->batch * p->x * p->n, p->k,
                                                 packmap(p), true, as_stream(stream)));
    return hip_status(gfft::launch_pack(f64(p), src, dst, p->batch * p->p * p->x, p->lg_x,
                                        p->lg_p, p->n, p->y, p->k, true, as_stream(stream)));
}

gfft_status gfft_unpack_slab_from_alltoall(const gfft_plan* p, const void* src, void* dst,
                                           void* stream) {
    if (!p) return GFFT_E_INVALID_ARG;
    if (p->pencil) return pencil_pack(p, src, dst, false, stream);
    gfft_status st = check_ptr(src);
    if (st != GFFT_OK || (st = check_ptr(dst)) != GFFT_OK) return st;
    if (overlap(src, cplx_bytes(p), dst, cplx_bytes(p))) return GFFT_E_INVALID_ARG;
    if ((st = check_device(p)) != GFFT_OK) return st;
    if (paper(p))
        return hip_status(gfft::launch_pack_rows(f64(p), src, dst, p->batch * p->x * p->n, p->k,
                                                 packmap(p), false, as_stream(stream)));
    return hip_status(gfft::launch_pack(f64(p), src, dst, p->batch * p->p * p->x, p->lg_x,
                                        p->lg_p, p->n, p->y, p->k, false, as_stream(stream)));
}

gfft_status gfft_exec_x_c2c(const gfft_plan* p, void* pencil, int sign, void* stream) {
    if (!p) return GFFT_E_INVALID_ARG;
    if (sign != -1 && sign != 1) return GFFT_E_INVALID_ARG;
    gfft_status st = check_ptr(pencil);
    if (st != GFFT_OK || (st = check_device(p)) != GFFT_OK) return st;
    return run_x(p, pencil, sign, as_stream(stream));
}

gfft_status gfft_exec_z_r2c(const gfft_plan* p, const void* in, void* out, double scale,
                            int weighted, void* stream) {
    gfft_status st = check_r2c_args(p, in, out);
    if (st != GFFT_OK) return st;
    if (!std::isfinite(scale)) return GFFT_E_INVALID_ARG;
    if ((st = check_device(p)) != GFFT_OK) return st;
    return run_z_r2c(p, in, out, scale, weighted != 0, as_stream(stream));
}

gfft_status gfft_exec_y_c2c(const gfft_plan* p, void* data, int sign, void* stream) {
    if (!p) return GFFT_E_INVALID_ARG;
    if (sign != -1 && sign != 1) return GFFT_E_INVALID_ARG;
    gfft_status st = check_ptr(data);
    if (st != GFFT_OK || (st = check_device(p)) != GFFT_OK) return st;
    return run_y(p, data, sign, as_stream(stream));
}

gfft_status gfft_exec_z_c2r(const gfft_plan* p, const void* in, void* out, double scale,
                            int weighted, void* stream) {
    gfft_status st = check_r2c_args(p, out, in);
    if (st != GFFT_OK) return st;
    if (!std::isfinite(scale)) return GFFT_E_INVALID_ARG;
    if ((st = check_device(p)) != GFFT_OK) return st;
    return run_z_c2r(p, in, out, scale, weighted != 0, as_stream(stream));
}

gfft_status gfft_exec_pass_copy(const gfft_plan* p, int axis, void* data, void* stream) {
    if (!p) return GFFT_E_INVALID_ARG;
    if (axis != 0 && axis != 1) return GFFT_E_INVALID_ARG;
    gfft_status st = check_ptr(data);
    if (st != GFFT_OK || (st = check_device(p)) != GFFT_OK) return st;
    return axis == 0 ? run_y(p, data, -1, as_stream(stream), true)
                     : run_x(p, data, -1, as_stream(stream), true);
}

gfft_status gfft_device_copy(void* dst, const void* src, int64_t bytes, void* stream) {
    if (bytes < 0 || bytes % 16 != 0) return GFFT_E_INVALID_ARG;
    gfft_status st = check_ptr(src);
    if (st != GFFT_OK || (st = check_ptr(dst)) != GFFT_OK) return st;
    if (overlap(src, bytes, dst, bytes)) return GFFT_E_INVALID_ARG;
    if (bytes == 0) return GFFT_OK;
    return hip_status(gfft::launch_copy16(src, dst, bytes / 16, as_stream(stream)));
}

}  // extern "C"
