// HIP kernels (gfx950) for the OMPDart data-flow solve.
//
// ompd_k_prep  (one 256-thread workgroup per CFG): ingest and normalise —
//   validates the CSR and the boundary rules, builds the predecessor CSR
//   (with the successor-edge id of every predecessor link), assigns every
//   block a level = longest path from a level-0 block over forward edges
//   (u -> v with u < v), and bucket-sorts blocks by level.
//
// ompd_k_solve (persistent, one wavefront per tile): a tile is one CFG and a
//   range of bit-slices (8, 16 or 32 variables per slice).  The tile runs
//   every phase of the method on its variables:
//     next use (backward may), validity with eager copies (forward must),
//     pending copies (forward may), delayed placement (forward AND/OR) and
//     its materialisation, validity after placement (forward must), the
//     reachability facts behind the map/update labels, and the per-variable
//     map kind (Table II).
//   Each phase iterates Gauss-Seidel sweeps over the levels: within a level
//   the 64 lanes evaluate (block, slice) items in parallel, levels go in
//   order (reverse order for the backward phase), and the iterated vector
//   of the phase stays in LDS.  A sweep that changes nothing ends the phase
//   (wavefront vote); every phase is monotone on a finite lattice, so the
//   chaotic order reaches the unique fixed point and the result does not
//   depend on the schedule.
//
// All arithmetic is integer AND / OR / ANDN; variables never interact, so
// any slicing of the variable axis is exact.
#include <hip/hip_runtime.h>

#include "ompd_device.h"

#define OMPD_E_INVAL_ (-1)
#define OMPD_E_NOCONVERGE_ (-4)

namespace ompd {

__device__ __forceinline__ void set_status(int32_t* info, int32_t code)
{
    atomicCAS(&info[INFO_STATUS], 0, code);
}

// Inclusive prefix sum of a[0..n) in global memory by one workgroup.
__device__ void block_scan_inclusive(int32_t* a, int n, int32_t* sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int carry = 0;
    for (int base = 0; base < n; base += blockDim.x) {
        int i = base + threadIdx.x;
        int x = (i < n) ? a[i] : 0;
        for (int d = 1; d < 64; d <<= 1) {
            int y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) sh[wv] = x;
        __syncthreads();
        int off = carry, tot = 0;
        for (int j = 0; j < nw; ++j) {
            if (j < wv) off += sh[j];
            tot += sh[j];
        }
        __syncthreads();
        if (i < n) a[i] = x + off;
        carry += tot;
    }
    __syncthreads();
}

// --------------------------------------------------------------------------
// ingest / normalise
// --------------------------------------------------------------------------
extern "C" __global__ void __launch_bounds__(256)
ompd_k_prep(const DevCfg* __restrict__ cfgs, int n_cfgs, int32_t* __restrict__ solve_counter)
{
    extern __shared__ __align__(16) int32_t plds[];
    __shared__ int s_err;
    __shared__ int s_max;
    __shared__ int32_t s_scan[16];
    const int ci = blockIdx.x;
    if (ci == 0 && threadIdx.x == 0) *solve_counter = 0;
    if (ci >= n_cfgs) return;
    const DevCfg c = cfgs[ci];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nb = c.nb, ne = c.ne, wd = c.wd;
    if (tid == 0) { s_err = 0; s_max = 0; }
    for (int i = tid; i < INFO_WORDS; i += nt) c.info[i] = 0;
    __syncthreads();

    // validation, stage 1: pointers, kinds, spaces
    int err = 0;
    if (tid == 0 && (c.succ_ptr[0] != 0 || c.succ_ptr[nb] != ne)) err = 1;
    for (int b = tid; b < nb; b += nt) {
        int a = c.succ_ptr[b], z = c.succ_ptr[b + 1];
        if (z < a || a < 0 || z > ne) err = 1;
        if (c.space[b] > 1) err = 1;
    }
    for (int e = tid; e < ne; e += nt)
        if (c.kind[e] > 2) err = 1;
    if (tid == 0 && (c.space[c.entry] != 0 || c.space[c.exit] != 0)) err = 1;
    if (err) atomicOr(&s_err, 1);
    __syncthreads();
    if (s_err) { if (tid == 0) c.info[INFO_STATUS] = OMPD_E_INVAL_; return; }

    // stage 2: successor targets, ENTRY/EXIT rules, bit rows, boundaries, calls
    if (tid == 0 && c.succ_ptr[c.exit + 1] != c.succ_ptr[c.exit]) err = 1;
    for (int e = tid; e < ne; e += nt) {
        int q = c.succ_idx[e];
        if (q < 0 || q >= nb || q == c.entry) err = 1;
        else if (q == c.exit && c.kind[e] != 0) err = 1;
    }
    for (int e = c.succ_ptr[c.entry] + tid; e < c.succ_ptr[c.entry + 1]; e += nt)
        if (c.kind[e] == 1) err = 1;
    if (wd > 0) {
        const uint64_t last = (c.nv & 63) ? ((1ull << (c.nv & 63)) - 1ull) : ~0ull;
        for (int w = tid; w < wd; w += nt) {
            uint64_t m = (w == wd - 1) ? last : ~0ull;
            if (c.R[(size_t)c.entry * wd + w] | c.W[(size_t)c.entry * wd + w] |
                c.R[(size_t)c.exit * wd + w] | c.W[(size_t)c.exit * wd + w]) err = 1;
            uint64_t eh = c.ev_h[w], ed = c.ev_d[w];
            if ((eh | ed | c.lx_h[w] | c.lx_d[w]) & ~m) err = 1;
            if (((eh | ed) & m) != m) err = 1;
        }
        for (int b = tid; b < nb; b += nt)
            if ((c.R[(size_t)b * wd + wd - 1] | c.W[(size_t)b * wd + wd - 1]) & ~last) err = 1;
    }
    if (c.call) {
        for (int b = tid; b < nb; b += nt) {
            int k = c.call[b];
            if (k >= 0 && (k >= c.n_sums || c.space[b] != 0 || b == c.entry || b == c.exit)) err = 1;
        }
    }
    if (err) atomicOr(&s_err, 1);
    __syncthreads();
    if (s_err) { if (tid == 0) c.info[INFO_STATUS] = OMPD_E_INVAL_; return; }

    // predecessor CSR
    int32_t* pp = c.pred_ptr;
    for (int b = tid; b <= nb; b += nt) pp[b] = 0;
    __syncthreads();
    for (int e = tid; e < ne; e += nt) atomicAdd(&pp[c.succ_idx[e] + 1], 1);
    __syncthreads();
    block_scan_inclusive(pp + 1, nb, s_scan);
    for (int b = tid; b < nb; b += nt) c.tmp[b] = pp[b];
    __syncthreads();
    for (int b = tid; b < nb; b += nt)
        for (int e = c.succ_ptr[b]; e < c.succ_ptr[b + 1]; ++e) {
            int q = c.succ_idx[e];
            int pos = atomicAdd(&c.tmp[q], 1);
            c.pred_idx[pos] = b;
            c.pred_eid[pos] = e;
        }
    __syncthreads();

    // levels: longest path over forward edges, chunk by chunk in id order;
    // inside a chunk, Jacobi rounds until no level changes
    int32_t* lvl = plds;
    for (int c0 = 0; c0 < nb; c0 += nt) {
        const int b = c0 + tid;
        const bool act = b < nb;
        int a = act ? pp[b] : 0, z = act ? pp[b + 1] : 0;
        int f0 = -1, f1 = -1, f2 = -1, f3 = -1, nf = 0, extra = 0;
        for (int j = a; j < z; ++j) {
            int p = c.pred_idx[j];
            if (p >= b) continue;
            if (nf == 0) f0 = p; else if (nf == 1) f1 = p; else if (nf == 2) f2 = p; else if (nf == 3) f3 = p; else extra = 1;
            ++nf;
        }
        if (act) lvl[b] = 0;
        __syncthreads();
        for (;;) {
            int L = 0;
            if (act) {
                if (f0 >= 0) L = max(L, lvl[f0] + 1);
                if (f1 >= 0) L = max(L, lvl[f1] + 1);
                if (f2 >= 0) L = max(L, lvl[f2] + 1);
                if (f3 >= 0) L = max(L, lvl[f3] + 1);
                if (extra)
                    for (int j = a; j < z; ++j) {
                        int p = c.pred_idx[j];
                        if (p < b) L = max(L, lvl[p] + 1);
                    }
            }
            int ch = act && (L != lvl[b]);
            __syncthreads();
            if (ch) lvl[b] = L;
            if (!__syncthreads_or(ch)) break;
        }
    }
    int mx = 0;
    for (int b = tid; b < nb; b += nt) mx = max(mx, lvl[b]);
    atomicMax(&s_max, mx);
    __syncthreads();
    const int nL = s_max + 1;
    int32_t* hist = c.tmp;   // free again after the predecessor scatter; nL <= nb
    for (int l = tid; l < nL; l += nt) hist[l] = 0;
    __syncthreads();
    for (int b = tid; b < nb; b += nt) atomicAdd(&hist[lvl[b]], 1);
    __syncthreads();
    for (int l = tid; l < nL; l += nt) c.level_ptr[l + 1] = hist[l];
    if (tid == 0) c.level_ptr[0] = 0;
    __syncthreads();
    block_scan_inclusive(c.level_ptr + 1, nL, s_scan);
    for (int l = tid; l < nL; l += nt) hist[l] = c.level_ptr[l];
    __syncthreads();
    for (int b = tid; b < nb; b += nt) {
        int pos = atomicAdd(&hist[lvl[b]], 1);
        c.level_blk[pos] = b;
    }
    if (tid == 0) c.info[INFO_NLEVELS] = nL;
}

// --------------------------------------------------------------------------
// solve
// --------------------------------------------------------------------------
template <typename T>
struct Tv {
    const DevCfg& c;
    int s0, RW;
    __device__ __forceinline__ size_t row(int b, int k) const { return (size_t)b * RW + s0 + k; }
    __device__ __forceinline__ T ld(const uint64_t* p, int b, int k) const
    {
        return reinterpret_cast<const T*>(p)[row(b, k)];
    }
    __device__ __forceinline__ void st(uint64_t* p, int b, int k, T v) const
    {
        reinterpret_cast<T*>(p)[row(b, k)] = v;
    }
    __device__ __forceinline__ T vec(const uint64_t* p, int k) const
    {
        return reinterpret_cast<const T*>(p)[s0 + k];
    }
    __device__ __forceinline__ T sum(int ci, int r, int k) const
    {
        return reinterpret_cast<const T*>(c.sums)[((size_t)ci * SUM_ROWS + r) * RW + s0 + k];
    }
};

template <typename T>
__device__ __forceinline__ T ones() { return (T)~(T)0; }

template <typename T>
__device__ bool solve_tile(const DevCfg& c, int s0, int ns, uint8_t* lds)
{
    constexpr int BITS = 8 * (int)sizeof(T);
    const int lane = threadIdx.x;
    const int nb = c.nb;
    const int RW = c.wd * (64 / BITS);
    const int nsi = ns > 0 ? ns : 1;
    const int lg = 31 - __clz(nsi);          // nsi is a power of two
    const bool data = ns > 0;
    T* SH = reinterpret_cast<T*>(lds);
    T* SD = SH + (size_t)nb * nsi;
    uint8_t* FL = lds + ((2 * (size_t)nb * nsi * sizeof(T) + 15) & ~(size_t)15);
    uint32_t* ACC = reinterpret_cast<uint32_t*>(FL + ((nb + 15) & ~15));
    const int nL = c.info[INFO_NLEVELS];
    const int32_t* __restrict__ lp = c.level_ptr;
    const int32_t* __restrict__ lb = c.level_blk;
    const int32_t* __restrict__ sp = c.succ_ptr;
    const int32_t* __restrict__ si = c.succ_idx;
    const int32_t* __restrict__ pp = c.pred_ptr;
    const int32_t* __restrict__ pi = c.pred_idx;
    const int32_t* __restrict__ pe = c.pred_eid;
    const uint8_t* __restrict__ kind = c.kind;
    const uint8_t* __restrict__ space = c.space;
    const Tv<T> tv{c, s0, RW};
    const int cap = c.sweep_cap > 0 ? c.sweep_cap : 2 * nb + 2;

    auto vmask = [&](int k) -> T {
        long lo = (long)(s0 + k) * BITS;
        if (lo + BITS <= c.nv) return ones<T>();
        if (lo >= c.nv) return (T)0;
        return (T)((1u << (unsigned)(c.nv - lo)) - 1u);
    };
    auto is_call = [&](int b) -> int { return c.call ? c.call[b] : -1; };
    // USE_s(b): a read in block b when b lies in space s; at EXIT the liveness after the region
    auto use = [&](int s, int b, int k) -> T {
        if (b == c.exit) return tv.vec(s ? c.lx_d : c.lx_h, k);
        T r = tv.ld(c.R, b, k);
        return ((int)space[b] == s) ? r : (T)0;
    };
    // USE'_s(b): call blocks whose callee may touch the variable stop pending copies like a read
    auto use_stop = [&](int s, int b, int k) -> T {
        T u = use(s, b, k);
        int ci = is_call(b);
        if (ci >= 0)
            u |= tv.sum(ci, s ? SUM_MAYR_D : SUM_MAYR_H, k) | tv.sum(ci, SUM_MAYW_H, k) | tv.sum(ci, SUM_MAYW_D, k);
        return u;
    };
    auto wr = [&](int s, int b, int k) -> T {
        if (b == c.exit) return (T)0;
        return ((int)space[b] == s) ? tv.ld(c.W, b, k) : (T)0;
    };
    // validity transfer of a block (write here: valid here; write in the other space: stale here)
    auto valid_out = [&](int s, int b, int k, T in) -> T {
        T w = (b == c.exit) ? (T)0 : tv.ld(c.W, b, k);
        T a1 = ((int)space[b] == s) ? (T)(in | w) : (T)(in & ~w);
        int ci = is_call(b);
        if (ci >= 0) {
            const uint64_t* nus = s ? c.nu_d : c.nu_h;
            T l = 0;
            for (int e = sp[b]; e < sp[b + 1]; ++e) l |= tv.ld(nus, si[e], k);
            int base = s ? SUM_TD : SUM_TH;
            T t00 = tv.sum(ci, base + 0, k), t01 = tv.sum(ci, base + 1, k);
            T t10 = tv.sum(ci, base + 2, k), t11 = tv.sum(ci, base + 3, k);
            a1 = (T)((~a1 & ~l & t00) | (~a1 & l & t01) | (a1 & ~l & t10) | (a1 & l & t11));
        }
        return (T)(a1 & vmask(k));
    };

    // sweep driver: forward (levels ascending) or backward (descending)
    auto run_phase = [&](int phase, bool backward, auto&& item) -> bool {
        int sweeps = 0;
        for (;;) {
            bool changed = false;
            for (int li = 0; li < nL; ++li) {
                const int l = backward ? (nL - 1 - li) : li;
                const int a = lp[l];
                const int n = (lp[l + 1] - a) << lg;
                for (int i = lane; i < n; i += 64) {
                    const int b = lb[a + (i >> lg)];
                    const int k = i & (nsi - 1);
                    changed |= item(b, k);
                }
            }
            ++sweeps;
            if (__ballot(changed) == 0ull) break;
            if (sweeps >= cap) {
                if (lane == 0) set_status(c.info, OMPD_E_NOCONVERGE_);
                return false;
            }
        }
        if (lane == 0) atomicMax(&c.info[INFO_SWEEPS + phase], sweeps);
        return true;
    };
    auto for_all_items = [&](auto&& f) {
        const int n = nb << lg;
        for (int i = lane; i < n; i += 64) f(i >> lg, i & (nsi - 1));
    };
    auto sidx = [&](int b, int k) -> size_t { return ((size_t)b << lg) + k; };

    // ---------------------------------------------------------------- init
    for (int i = lane; i < (nb << lg); i += 64) { SH[i] = 0; SD[i] = 0; }
    for (int b = lane; b < nb; b += 64) {
        int dev = space[b] ? 1 : 0;
        FL[b] = (uint8_t)((b == c.exit ? 1 : 0) | (dev << 1) | (b == c.entry ? 4 : 0) | (dev << 3));
    }
    for (int i = lane; i < 3 * nsi; i += 64) ACC[i] = 0;
    __syncthreads();

    // ---------------------------------------------------------------- next use (backward, may)
    // NUin_s(b) = USE_s(b) | (NUout_s(b) & ~W_b), NUout_s = OR over successors.
    // Flags bits 0/1: reaches EXIT / reaches a DEVICE block (before_dev).
    if (!run_phase(PH_NU, true, [&](int b, int k) -> bool {
            bool ch = false;
            if (data) {
                T oH = 0, oD = 0;
                for (int e = sp[b]; e < sp[b + 1]; ++e) {
                    int q = si[e];
                    oH |= SH[sidx(q, k)];
                    oD |= SD[sidx(q, k)];
                }
                T vH, vD;
                if (b == c.exit) {
                    vH = tv.vec(c.lx_h, k);
                    vD = tv.vec(c.lx_d, k);
                } else {
                    T r = tv.ld(c.R, b, k), w = tv.ld(c.W, b, k);
                    T uH = space[b] ? (T)0 : r, uD = space[b] ? r : (T)0;
                    int ci = is_call(b);
                    if (ci >= 0) {
                        vH = uH | (~w & (tv.sum(ci, SUM_NU0_H, k) | (tv.sum(ci, SUM_NU1_H, k) & oH)));
                        vD = uD | (~w & (tv.sum(ci, SUM_NU0_D, k) | (tv.sum(ci, SUM_NU1_D, k) & oD)));
                    } else {
                        vH = uH | (oH & ~w);
                        vD = uD | (oD & ~w);
                    }
                }
                T m = vmask(k);
                vH &= m; vD &= m;
                size_t li = sidx(b, k);
                if (vH != SH[li]) { SH[li] = vH; ch = true; }
                if (vD != SD[li]) { SD[li] = vD; ch = true; }
            }
            if (k == 0) {
                uint8_t f = FL[b], g = 0;
                for (int e = sp[b]; e < sp[b + 1]; ++e) g |= FL[si[e]];
                uint8_t nf = (uint8_t)(f | (g & 3));
                if (nf != f) { FL[b] = nf; ch = true; }
            }
            return ch;
        }))
        return false;
    if (data)
        for_all_items([&](int b, int k) {
            tv.st(c.nu_h, b, k, SH[sidx(b, k)]);
            tv.st(c.nu_d, b, k, SD[sidx(b, k)]);
        });
    __syncthreads();

    // ---------------------------------------------------------------- validity with eager copies
    // AVEin_s(q) = NUin_s(q) | AND over preds AVEout_s(p); AVEin(ENTRY) = boundary.
    // Flags bits 2/3: reached from ENTRY / reached from a DEVICE block (after_dev).
    auto ave_in = [&](int q, int k, T& iH, T& iD) {
        if (q == c.entry) {
            iH = tv.vec(c.ev_h, k);
            iD = tv.vec(c.ev_d, k);
        } else {
            T mH = ones<T>(), mD = ones<T>();
            for (int j = pp[q]; j < pp[q + 1]; ++j) {
                int p = pi[j];
                mH &= SH[sidx(p, k)];
                mD &= SD[sidx(p, k)];
            }
            iH = tv.ld(c.nu_h, q, k) | mH;
            iD = tv.ld(c.nu_d, q, k) | mD;
        }
        T m = vmask(k);
        iH &= m; iD &= m;
    };
    for (int i = lane; i < (nb << lg); i += 64) { SH[i] = ones<T>(); SD[i] = ones<T>(); }
    if (!run_phase(PH_AVE, false, [&](int q, int k) -> bool {
            bool ch = false;
            if (data) {
                T iH, iD;
                ave_in(q, k, iH, iD);
                T oH = valid_out(0, q, k, iH), oD = valid_out(1, q, k, iD);
                size_t li = sidx(q, k);
                if (oH != SH[li]) { SH[li] = oH; ch = true; }
                if (oD != SD[li]) { SD[li] = oD; ch = true; }
            }
            if (k == 0) {
                uint8_t f = FL[q], g = 0;
                for (int j = pp[q]; j < pp[q + 1]; ++j) g |= FL[pi[j]];
                uint8_t nf = (uint8_t)(f | (g & 12));
                if (nf != f) { FL[q] = nf; ch = true; }
            }
            return ch;
        }))
        return false;
    if (data)
        for_all_items([&](int q, int k) {
            T iH, iD;
            ave_in(q, k, iH, iD);
            tv.st(c.ave_h, q, k, iH);
            tv.st(c.ave_d, q, k, iD);
            tv.st(c.aveout_h, q, k, SH[sidx(q, k)]);
            tv.st(c.aveout_d, q, k, SD[sidx(q, k)]);
        });
    {
        bool bad = false;
        for (int b = lane; b < nb; b += 64) {
            uint8_t f = FL[b];
            if ((f & 5) != 5) bad = true;
            if (s0 == 0) {
                if (c.after_dev) c.after_dev[b] = (f >> 3) & 1;
                if (c.before_dev) c.before_dev[b] = (f >> 1) & 1;
            }
        }
        if (__ballot(bad) != 0ull) {
            if (lane == 0) set_status(c.info, OMPD_E_INVAL_);
            return false;
        }
    }
    __syncthreads();

    // EAG_s(e=p->q) = NUin_s(q) & ~AVEout_s(p)
    if (c.placement == 0) {
        // ------------------------------------------------------------ pending copies (forward, may)
        // MAYP_s(e) = (EAG_s(e) | MAYPout_s(p)) & ~LE(e); MAYPout_s(q) = OR_e MAYP_s(e) & ~USE'_s(q) & ~WR_s(q)
        for (int i = lane; i < (nb << lg); i += 64) { SH[i] = 0; SD[i] = 0; }
        if (data) {
            if (!run_phase(PH_MAYP, false, [&](int q, int k) -> bool {
                    if (q == c.entry) return false;
                    T nuH = tv.ld(c.nu_h, q, k), nuD = tv.ld(c.nu_d, q, k);
                    T mH = 0, mD = 0;
                    for (int j = pp[q]; j < pp[q + 1]; ++j) {
                        int p = pi[j];
                        T nle = (kind[pe[j]] == 2) ? (T)0 : ones<T>();
                        T aH = tv.ld(c.aveout_h, p, k), aD = tv.ld(c.aveout_d, p, k);
                        mH |= ((nuH & ~aH) | SH[sidx(p, k)]) & nle;
                        mD |= ((nuD & ~aD) | SD[sidx(p, k)]) & nle;
                    }
                    T m = vmask(k);
                    T vH = mH & ~use_stop(0, q, k) & ~wr(0, q, k) & m;
                    T vD = mD & ~use_stop(1, q, k) & ~wr(1, q, k) & m;
                    bool ch = false;
                    size_t li = sidx(q, k);
                    if (vH != SH[li]) { SH[li] = vH; ch = true; }
                    if (vD != SD[li]) { SD[li] = vD; ch = true; }
                    return ch;
                }))
                return false;
            for_all_items([&](int q, int k) {
                tv.st(c.mayp_h, q, k, SH[sidx(q, k)]);
                tv.st(c.mayp_d, q, k, SD[sidx(q, k)]);
            });
        }
        __syncthreads();

        // ------------------------------------------------------------ delayed placement (forward, LFP)
        // LATER_s(e) = EAG_s(e) | LATERout_s(p); L'_s(e) = LATER_s(e) & ~LE(e)
        // FV_x(e) = (AVEout_x(p) | EAG_x(e)) & ~MAYP_x(e)
        // N'_s(e) = (FV_s(e) & FV_o(e)) | (LATER_s(e) & LE(e))
        // LATERin_s(q) = AND_e (L'_s | N'_s) & OR_e L'_s; LATERout_s(q) = LATERin_s(q) & ~USE'_s(q) & ~WR_s(q)
        auto later_in = [&](int q, int k, T& lH, T& lD) {
            T nuH = tv.ld(c.nu_h, q, k), nuD = tv.ld(c.nu_d, q, k);
            T allH = ones<T>(), allD = ones<T>(), anyH = 0, anyD = 0;
            for (int j = pp[q]; j < pp[q + 1]; ++j) {
                int p = pi[j];
                T le = (kind[pe[j]] == 2) ? ones<T>() : (T)0;
                T aH = tv.ld(c.aveout_h, p, k), aD = tv.ld(c.aveout_d, p, k);
                T mpH = tv.ld(c.mayp_h, p, k), mpD = tv.ld(c.mayp_d, p, k);
                T eH = nuH & ~aH, eD = nuD & ~aD;
                T fvH = (aH | eH) & ~((eH | mpH) & ~le);
                T fvD = (aD | eD) & ~((eD | mpD) & ~le);
                T latH = eH | SH[sidx(p, k)], latD = eD | SD[sidx(p, k)];
                T lpH = latH & ~le, lpD = latD & ~le;
                T both = fvH & fvD;
                allH &= lpH | both | (latH & le);
                allD &= lpD | both | (latD & le);
                anyH |= lpH;
                anyD |= lpD;
            }
            T m = vmask(k);
            lH = allH & anyH & m;
            lD = allD & anyD & m;
        };
        for (int i = lane; i < (nb << lg); i += 64) { SH[i] = 0; SD[i] = 0; }
        if (data) {
            if (!run_phase(PH_LATER, false, [&](int q, int k) -> bool {
                    if (q == c.entry) return false;
                    T lH, lD;
                    later_in(q, k, lH, lD);
                    T vH = lH & ~use_stop(0, q, k) & ~wr(0, q, k);
                    T vD = lD & ~use_stop(1, q, k) & ~wr(1, q, k);
                    bool ch = false;
                    size_t li = sidx(q, k);
                    if (vH != SH[li]) { SH[li] = vH; ch = true; }
                    if (vD != SD[li]) { SD[li] = vD; ch = true; }
                    return ch;
                }))
                return false;
            // materialise: INS_ENTRY_s(q) = LATERin_s(q) & USE'_s(q);
            //              INS_EDGE_s(e=p->q) = LATER_s(e) & (LE(e) | ~LATERin_s(q))
            for_all_items([&](int q, int k) {
                T lH = 0, lD = 0;
                if (q != c.entry) later_in(q, k, lH, lD);
                tv.st(c.ie_h, q, k, lH & use_stop(0, q, k));
                tv.st(c.ie_d, q, k, lD & use_stop(1, q, k));
                T nuH = tv.ld(c.nu_h, q, k), nuD = tv.ld(c.nu_d, q, k);
                T m = vmask(k);
                for (int j = pp[q]; j < pp[q + 1]; ++j) {
                    int p = pi[j], e = pe[j];
                    T le = (kind[e] == 2) ? ones<T>() : (T)0;
                    T latH = (nuH & ~tv.ld(c.aveout_h, p, k)) | SH[sidx(p, k)];
                    T latD = (nuD & ~tv.ld(c.aveout_d, p, k)) | SD[sidx(p, k)];
                    tv.st(c.ig_h, e, k, latH & (le | ~lH) & m);
                    tv.st(c.ig_d, e, k, latD & (le | ~lD) & m);
                }
            });
        }
    } else if (data) {
        // eager placement only: every EAG is materialised on its edge
        for_all_items([&](int q, int k) {
            tv.st(c.ie_h, q, k, (T)0);
            tv.st(c.ie_d, q, k, (T)0);
            T nuH = tv.ld(c.nu_h, q, k), nuD = tv.ld(c.nu_d, q, k);
            T m = vmask(k);
            for (int j = pp[q]; j < pp[q + 1]; ++j) {
                int p = pi[j], e = pe[j];
                tv.st(c.ig_h, e, k, nuH & ~tv.ld(c.aveout_h, p, k) & m);
                tv.st(c.ig_d, e, k, nuD & ~tv.ld(c.aveout_d, p, k) & m);
            }
        });
    }
    __syncthreads();

    // ---------------------------------------------------------------- validity after placement
    // AVFin_s(q) = INS_ENTRY_s(q) | AND_e (AVFout_s(p) | INS_EDGE_s(e))
    auto avf_in = [&](int q, int k, T& iH, T& iD) {
        if (q == c.entry) {
            iH = tv.vec(c.ev_h, k);
            iD = tv.vec(c.ev_d, k);
        } else {
            T mH = ones<T>(), mD = ones<T>();
            for (int j = pp[q]; j < pp[q + 1]; ++j) {
                int p = pi[j], e = pe[j];
                mH &= SH[sidx(p, k)] | tv.ld(c.ig_h, e, k);
                mD &= SD[sidx(p, k)] | tv.ld(c.ig_d, e, k);
            }
            iH = tv.ld(c.ie_h, q, k) | mH;
            iD = tv.ld(c.ie_d, q, k) | mD;
        }
        T m = vmask(k);
        iH &= m; iD &= m;
    };
    if (data) {
        for (int i = lane; i < (nb << lg); i += 64) { SH[i] = ones<T>(); SD[i] = ones<T>(); }
        if (!run_phase(PH_AVF, false, [&](int q, int k) -> bool {
                T iH, iD;
                avf_in(q, k, iH, iD);
                T oH = valid_out(0, q, k, iH), oD = valid_out(1, q, k, iD);
                bool ch = false;
                size_t li = sidx(q, k);
                if (oH != SH[li]) { SH[li] = oH; ch = true; }
                if (oD != SD[li]) { SD[li] = oD; ch = true; }
                return ch;
            }))
            return false;
        // outputs, and the per-variable map kind (Table II):
        // map(to) copy into D: on p->q with !after_dev(p), before q with no after_dev predecessor;
        // map(from) copy into H: on p->q or before q with !before_dev(q).
        for_all_items([&](int q, int k) {
            if (c.avf_h) {
                T iH, iD;
                avf_in(q, k, iH, iD);
                tv.st(c.avf_h, q, k, iH);
                tv.st(c.avf_d, q, k, iD);
            }
            if (c.var_kind) {
                T to = 0, from = 0, dev = 0;
                const bool before_q = (FL[q] >> 1) & 1;
                bool pred_after = false;
                for (int j = pp[q]; j < pp[q + 1]; ++j) {
                    int p = pi[j], e = pe[j];
                    bool after_p = (FL[p] >> 3) & 1;
                    pred_after |= after_p;
                    if (!after_p) to |= tv.ld(c.ig_d, e, k);
                    if (!before_q) from |= tv.ld(c.ig_h, e, k);
                }
                if (!pred_after) to |= tv.ld(c.ie_d, q, k);
                if (!before_q) from |= tv.ld(c.ie_h, q, k);
                if (space[q] && q != c.exit) dev = tv.ld(c.R, q, k) | tv.ld(c.W, q, k);
                if (to) atomicOr(&ACC[k], (uint32_t)to);
                if (from) atomicOr(&ACC[nsi + k], (uint32_t)from);
                if (dev) atomicOr(&ACC[2 * nsi + k], (uint32_t)dev);
            }
        });
        __syncthreads();
        if (c.var_kind) {
            for (int v = lane; v < ns * BITS; v += 64) {
                long gv = (long)s0 * BITS + v;
                if (gv >= c.nv) continue;
                int k = v / BITS, bit = v % BITS;
                uint32_t to = (ACC[k] >> bit) & 1u, from = (ACC[nsi + k] >> bit) & 1u, dv = (ACC[2 * nsi + k] >> bit) & 1u;
                c.var_kind[gv] = (uint8_t)(to | (from << 1) | ((dv && !to && !from) ? 4u : 0u));
            }
        }
    }
    return true;
}

extern "C" __global__ void __launch_bounds__(64)
ompd_k_solve(const DevCfg* __restrict__ cfgs, const Tile* __restrict__ tiles, int n_tiles, int32_t* __restrict__ counter)
{
    extern __shared__ __align__(16) uint8_t slds[];
    for (;;) {
        int t = 0;
        if (threadIdx.x == 0) t = atomicAdd(counter, 1);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
        if (t >= n_tiles) break;
        const Tile tl = tiles[t];
        const DevCfg c = cfgs[tl.cfg];
        if (c.info[INFO_STATUS] != 0) continue;
        if (tl.tbits == 32) solve_tile<uint32_t>(c, tl.s0, tl.ns, slds);
        else if (tl.tbits == 16) solve_tile<uint16_t>(c, tl.s0, tl.ns, slds);
        else solve_tile<uint8_t>(c, tl.s0, tl.ns, slds);
        __syncthreads();
    }
}

}  // namespace ompd
