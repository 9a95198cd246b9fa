// Context, batched device operators and the host control of the PNCG
// minimizer (Alg. 4 with beta*ZA, the local-field preconditioner solved by
// Alg. 1, and field stepping), behind the C ABI of include/mmncg.h.
//
// A context holds one or more independent problem instances. Their operators
// are concatenated (each instance padded to whole SELL slices) and every
// kernel launch serves all instances at once; each instance runs its own
// copy of the minimizer's control logic on the host. One "round" of the
// batched driver is
//   1. one batched evaluation (trial points of the line searches and start
//      points of new field values, including the scalar-potential solve),
//   2. host decisions per instance (line-search steps, acceptance, stopping),
//   3. one batched copy of accepted trials, preconditioner solve and
//      direction update for the instances that need a new direction.
// Instances advance through their field lists independently. The host only
// makes scalar decisions; every vector operation runs in the HIP kernels on
// the context's stream. Scalars come back through small pinned buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mmncg.h"
#include "internal.h"
#include "context.h"

using namespace mmncg;

namespace mmncg {

// ---------------------------------------------------------------------------
// plumbing
// ---------------------------------------------------------------------------
void *dalloc(mm_ctx *c, size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (c->ualloc) {
        p = c->ualloc(bytes, c->user);
        if (!p) throw ApiError{MM_ENOMEM, "device allocation callback failed"};
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw ApiError{MM_ENOMEM, "hipMalloc failed (" + std::to_string(bytes) + " bytes)"};
        }
    }
    c->allocs.push_back({p, bytes});
    c->dev_bytes += bytes;
    return p;
}
void dfree(mm_ctx *c, void *p) {
    if (!p) return;
    for (size_t k = 0; k < c->allocs.size(); ++k)
        if (c->allocs[k].first == p) {
            c->dev_bytes -= c->allocs[k].second;
            c->allocs.erase(c->allocs.begin() + (long)k);
            if (c->ufree) c->ufree(p, c->user);
            else (void)hipFree(p);
            return;
        }
}

void free_host_ctl(mm_ctx *c) {
    // hci lives in hcd's allocation (one copy uploads both)
    c->hci = nullptr;
    for (void **p : {(void **)&c->hcd, (void **)&c->hsc, (void **)&c->hpst, (void **)&c->hpr}) {
        if (*p) (void)hipHostFree(*p);
        *p = nullptr;
    }
}

void free_all(mm_ctx *c) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    amg_release(c);
    c->hostK.clear();
    for (hipGraphExec_t *g : {&c->graph64, &c->graph32, &c->agraph64, &c->mgraph}) {
        if (*g) (void)hipGraphExecDestroy(*g);
        *g = nullptr;
    }
    for (auto &a : c->allocs) {
        if (c->ufree) c->ufree(a.first, c->user);
        else (void)hipFree(a.first);
    }
    c->allocs.clear();
    c->dev_bytes = 0;
    free_host_ctl(c);
    c->ninst = 0;
    c->inst.clear();
}

bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

void copy_in(mm_ctx *c, double *dst, const double *src, size_t n) {
    if (n == 0) return;
    HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double),
                          is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
}
void pot_in(mm_ctx *c, double *dev, const double *abi, double *tmp) {
    const int n = c->inst[0].n_pot;
    copy_in(c, tmp, abi, n);
    launch_gather(n, c->pord, tmp, dev, c->stream);
}
void pot_out(mm_ctx *c, double *abi, const double *dev, double *tmp) {
    const int n = c->inst[0].n_pot;
    launch_gather(n, c->ppos, dev, tmp, c->stream);
    copy_out(c, abi, tmp, n);
}
void copy_out(mm_ctx *c, double *dst, const double *src, size_t n) {
    if (n == 0) return;
    HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double),
                          is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
}
void kt_harvest(mm_ctx *c);
void sync(mm_ctx *c) {
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->kt_on) kt_harvest(c);
}

// The host writes the control block only after a synchronization that
// follows the previous upload, so an upload never races with the host.
void upload_ctl(mm_ctx *c) {
    const int n = c->ninst;
    // the doubles and the first six int arrays are contiguous (see setup)
    HIPCHK(hipMemcpyAsync(c->dcd, c->hcd, 8 * (size_t)n * sizeof(double) + 6 * (size_t)n * sizeof(int),
                          hipMemcpyHostToDevice, c->stream));
}
void pull_flags(mm_ctx *c) {
    const int n = c->ninst;
    HIPCHK(hipMemcpyAsync(c->hci + 6 * n, c->dci + 6 * n, 5 * (size_t)n * sizeof(int), hipMemcpyDeviceToHost,
                          c->stream));
}
enum { SC_EVAL = 0, SC_DIR = kEvalParts, SC_MISC = kEvalParts + 2, SC_PER = kEvalParts + 7 };
double *dsc_at(mm_ctx *c, int slot) { return c->dsc + (size_t)slot * c->ninst; }
double *hsc_at(mm_ctx *c, int slot) { return c->hsc + (size_t)slot * c->ninst; }
// finalize output of slot group `slot` with `nq` quantities is [inst][nq]
void pull_sc(mm_ctx *c, int slot, int nq) {
    HIPCHK(hipMemcpyAsync(hsc_at(c, slot), dsc_at(c, slot), (size_t)nq * c->ninst * sizeof(double),
                          hipMemcpyDeviceToHost, c->stream));
}
double *mslot(mm_ctx *c, int q) { return c->mpart + (size_t)q * c->Mm.map.nblk; }

// event pairs around the timed kernels; harvested at the next synchronization
void prof_mark(mm_ctx *c) {
    if (!c->prof_on) return;
    if (c->prof_used == c->prof_ev.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        c->prof_ev.push_back(e);
    }
    HIPCHK(hipEventRecord(c->prof_ev[c->prof_used++], c->stream));
}
void prof_harvest(mm_ctx *c) {
    for (size_t i = 0; i + 1 < c->prof_used; i += 2) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, c->prof_ev[i], c->prof_ev[i + 1]));
        c->prof_seconds += ms * 1e-3;
    }
    c->prof_used = 0;
}

// field-kernel timers: an event before and after one launch (pair p of
// kernel k uses events 2p and 2p + 1), harvested after the next
// synchronization of the stream
void kt_begin(mm_ctx *c, int k) {
    if (!c->kt_on) return;
    std::vector<hipEvent_t> &ev = c->kt_ev[k];
    const size_t at = 2 * c->kt_pend[k].size();
    while (ev.size() < at + 2) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ev.push_back(e);
    }
    HIPCHK(hipEventRecord(ev[at], c->stream));
}
void kt_end(mm_ctx *c, int k, double bytes) {
    if (!c->kt_on) return;
    HIPCHK(hipEventRecord(c->kt_ev[k][2 * c->kt_pend[k].size() + 1], c->stream));
    c->kt_pend[k].push_back(bytes);
}
void kt_harvest(mm_ctx *c) {
    for (int k = 0; k < KT_N; ++k) {
        for (size_t p = 0; p < c->kt_pend[k].size(); ++p) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, c->kt_ev[k][2 * p], c->kt_ev[k][2 * p + 1]));
            c->kt_sec[k] += ms * 1e-3;
            c->kt_calls[k] += 1;
            c->kt_bytes[k] += c->kt_pend[k][p];
        }
        c->kt_pend[k].clear();
    }
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// operator concatenation and SELL-64 upload
// ---------------------------------------------------------------------------
// append instance operator h to the global G: rows from row_off (padding rows
// before it are empty), columns shifted by col_off, output rows by out_off
void append_csr(HostCsr &G, const HostCsr &h, int row_off, int col_off, int out_off) {
    if (G.ptr.empty()) G.ptr.push_back(0);
    G.vw = h.vw;
    const bool ro = !h.row_out.empty();
    while (G.nrows < row_off) {
        G.ptr.push_back(G.ptr.back());
        if (ro || !G.row_out.empty()) G.row_out.push_back(0);
        G.nrows++;
    }
    if (ro && G.row_out.size() < (size_t)G.nrows) G.row_out.resize(G.nrows, 0);
    for (int r = 0; r < h.nrows; ++r) {
        for (int64_t k = h.ptr[r]; k < h.ptr[r + 1]; ++k) {
            G.col.push_back(h.col[k] + col_off);
            for (int q = 0; q < h.vw; ++q) G.val.push_back(h.val[k * h.vw + q]);
        }
        G.ptr.push_back((int64_t)G.col.size());
        if (ro) G.row_out.push_back(h.row_out[r] + out_off);
        G.nrows++;
    }
}
void pad_rows(HostCsr &G, int nrows) {
    if (G.ptr.empty()) G.ptr.push_back(0);
    while (G.nrows < nrows) {
        G.ptr.push_back(G.ptr.back());
        if (!G.row_out.empty()) G.row_out.push_back(0);
        G.nrows++;
    }
}

// Padding entries of a slice point at a column that a real entry of the same
// slice uses (so they stay inside the instance) with value 0.
void upload_sell(mm_ctx *c, const HostCsr &h, Sell &d) {
    d.nrows = h.nrows;
    d.vw = h.vw;
    d.nslices = (h.nrows + kSlice - 1) / kSlice;
    std::vector<int64_t> sptr(d.nslices + 1, 0);
    std::vector<int> padc(d.nslices, 0);
    for (int s = 0; s < d.nslices; ++s) {
        int64_t w = 0;
        bool got = false;
        for (int r = s * kSlice; r < std::min(h.nrows, (s + 1) * kSlice); ++r) {
            w = std::max(w, h.ptr[r + 1] - h.ptr[r]);
            if (!got && h.ptr[r + 1] > h.ptr[r]) {
                padc[s] = h.col[h.ptr[r]];
                got = true;
            }
        }
        sptr[s + 1] = sptr[s] + w * kSlice;
    }
    d.padded = sptr[d.nslices];
    d.nnz = h.ptr.empty() ? 0 : h.ptr[h.nrows];
    std::vector<int> col(std::max<int64_t>(d.padded, 1), 0);
    std::vector<double> val(std::max<int64_t>(d.padded * h.vw, 1), 0.0);
    for (int s = 0; s < d.nslices; ++s) {
        const int64_t w = (sptr[s + 1] - sptr[s]) / kSlice;
        for (int ln = 0; ln < kSlice; ++ln) {
            int r = s * kSlice + ln;
            int64_t len = r < h.nrows ? h.ptr[r + 1] - h.ptr[r] : 0;
            for (int64_t k = 0; k < w; ++k) {
                int64_t e = sptr[s] + kSlice * k;
                if (k < len) {
                    col[e + ln] = h.col[h.ptr[r] + k];
                    for (int q = 0; q < h.vw; ++q)
                        val[e * h.vw + q * kSlice + ln] = h.val[(h.ptr[r] + k) * h.vw + q];
                } else {
                    col[e + ln] = padc[s];
                }
            }
        }
    }
    d.sptr = dalloc_n<int64_t>(c, sptr.size());
    d.col = dalloc_n<int>(c, col.size());
    d.val = dalloc_n<double>(c, val.size());
    d.val32 = dalloc_n<float>(c, val.size());
    HIPCHK(hipMemcpyAsync(d.sptr, sptr.data(), sptr.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(d.col, col.data(), col.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(d.val, val.data(), val.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    launch_to_f32((int64_t)val.size(), d.val, d.val32, c->stream);
    if (!h.row_out.empty()) {
        d.row_out = dalloc_n<int>(c, h.row_out.size());
        HIPCHK(hipMemcpyAsync(d.row_out, h.row_out.data(), h.row_out.size() * sizeof(int), hipMemcpyHostToDevice,
                              c->stream));
    }
    sync(c);  // host vectors go out of scope
}

void upload_vec(mm_ctx *c, double *dst, const std::vector<double> &v) {
    if (v.empty()) return;
    HIPCHK(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    sync(c);
}

// Partition of one row space into logical blocks: instance i owns rows
// [off[i], off[i] + n[i]) (off a multiple of 64); its ns = ceil(n/64) slices
// are split evenly over min(cap_i, ceil(ns / slices_per_block)) blocks, cap_i
// = 256, or one block per 8192 rows up to kMaxBlocksPerInst for very large
// instances, times cap_mult (the tuner's choice for the scalar-potential
// rows). With `fill`, cap_i = kMaxBlocksPerInst: the magnet-row kernels
// (4 waves per block, a few registers) need that many waves in flight to keep
// HBM busy on large instances, and their partials are few. The table is padded
// with empty blocks to a multiple of 8 (XCD renumbering).
void make_map(mm_ctx *c, DevMap &dm, const std::vector<int> &off, const std::vector<int> &n,
              const std::vector<int> &slices_per_block, bool fill = false, int cap_mult = 1) {
    const int ni = (int)off.size();
    std::vector<int> tab;
    std::vector<int> ipb(ni + 1, 0), rend(ni, 0);
    for (int i = 0; i < ni; ++i) {
        ipb[i] = (int)tab.size() / 4;
        const int ns = (n[i] + kSlice - 1) / kSlice;
        const int sf = off[i] / kSlice;
        rend[i] = off[i] + n[i];
        if (ns == 0) continue;
        const int spb = std::max(1, slices_per_block[i]);
        // at most 256 blocks per instance, more only for very large instances
        // (one per 8192 rows, up to kMaxBlocksPerInst): every block re-reduces
        // the instance's partials, which costs more than it gains below that
        const int cap = fill ? kMaxBlocksPerInst
                             : std::min(kMaxBlocksPerInst, cap_mult * std::max(256, (n[i] + 8191) / 8192));
        const int nb = std::min(cap, (ns + spb - 1) / spb);
        for (int k = 0; k < nb; ++k) {
            tab.push_back(i);
            tab.push_back(sf + (int)((int64_t)k * ns / nb));
            tab.push_back(sf + (int)((int64_t)(k + 1) * ns / nb));
            tab.push_back(0);
        }
    }
    ipb[ni] = (int)tab.size() / 4;
    while (tab.size() / 4 < 8 || (tab.size() / 4) % 8 != 0) {
        tab.push_back(-1);
        tab.push_back(0);
        tab.push_back(0);
        tab.push_back(0);
    }
    const int nblk = (int)tab.size() / 4;
    int4 *dtab = dalloc_n<int4>(c, nblk);
    int *dipb = dalloc_n<int>(c, ni + 1);
    int *drend = dalloc_n<int>(c, std::max(ni, 1));
    HIPCHK(hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dipb, ipb.data(), ipb.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(drend, rend.data(), rend.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    sync(c);
    dm.map.tab = dtab;
    dm.map.ipb = dipb;
    dm.map.rend = drend;
    dm.map.nblk = nblk;
    dm.map.ninst = ni;
}

int pad64(int n) { return (n + kSlice - 1) / kSlice * kSlice; }

// The local operators C and S in difference form (the device applies them as
// R_i x_i + sum_{j != i} A_ij (x_j - x_i)): the diagonal entry of every row
// takes the row sum R_i (per block component for C). A row without a stored
// diagonal is all zeros.
void to_difference_form(HostCsr &A) {
    const int vw = A.vw;
    for (int r = 0; r < A.nrows; ++r) {
        double sum[6] = {0, 0, 0, 0, 0, 0};
        int64_t dg = -1;
        for (int64_t e = A.ptr[r]; e < A.ptr[r + 1]; ++e) {
            for (int q = 0; q < vw; ++q) sum[q] += A.val[e * vw + q];
            if (A.col[e] == r) dg = e;
        }
        if (dg >= 0)
            for (int q = 0; q < vw; ++q) A.val[dg * vw + q] = sum[q];
    }
}

// A symmetric sparse matrix on renumbered rows: row r of the result is row
// ord[r] of A, column j becomes pos[j] (pos the inverse of ord)
HostCsr permute_sym(const HostCsr &A, const std::vector<int> &ord, const std::vector<int> &pos) {
    HostCsr P;
    P.nrows = A.nrows;
    P.vw = A.vw;
    P.ptr.assign(A.nrows + 1, 0);
    P.col.reserve(A.col.size());
    P.val.reserve(A.val.size());
    for (int r = 0; r < A.nrows; ++r) {
        const int a = ord[r];
        for (int64_t e = A.ptr[a]; e < A.ptr[a + 1]; ++e) {
            P.col.push_back(pos[A.col[e]]);
            for (int q = 0; q < A.vw; ++q) P.val.push_back(A.val[e * A.vw + q]);
        }
        P.ptr[r + 1] = (int64_t)P.col.size();
    }
    return P;
}

// Builds every device structure of a batch from the per-instance assemblies.
void setup_device(mm_ctx *c, std::vector<Assembly> &as, const std::vector<long> &nn, const std::vector<long> &nt) {
    free_all(c);
    const int ni = (int)as.size();
    c->ninst = ni;
    c->inst.assign(ni, InstInfo());
    std::vector<int> moff(ni), poff(ni), boff(ni), nm(ni), np(ni), nb(ni);
    int rm = 0, rp = 0, rb = 0;
    long uo = 0;
    for (int i = 0; i < ni; ++i) {
        InstInfo &I = c->inst[i];
        I.n_nodes = nn[i];
        I.n_tets = nt[i];
        I.n_mag = as[i].n_mag;
        I.n_pot = as[i].n_pot;
        I.n_brow = as[i].B.nrows;
        I.mag_off = moff[i] = rm;
        I.pot_off = poff[i] = rp;
        I.brow_off = boff[i] = rb;
        I.user_off = uo;
        I.nnz_C = as[i].C.ptr.empty() ? 0 : as[i].C.ptr[as[i].C.nrows];
        I.nnz_K = as[i].K.ptr.empty() ? 0 : as[i].K.ptr[as[i].K.nrows];
        I.nnz_B = as[i].B.ptr.empty() ? 0 : as[i].B.ptr[as[i].B.nrows];
        I.nnz_S = as[i].S.ptr.empty() ? 0 : as[i].S.ptr[as[i].S.nrows];
        I.Ms_ref = as[i].Ms_ref;
        I.node_of_mag = as[i].node_of_mag;
        nm[i] = I.n_mag;
        np[i] = I.n_pot;
        nb[i] = I.n_brow;
        rm += pad64(I.n_mag);
        rp += pad64(I.n_pot);
        rb += pad64(I.n_brow);
        uo += I.n_mag;
    }
    c->rows_m = rm;
    c->rows_p = rp;
    c->rows_b = rb;
    c->tot_mag = uo;
    {
        HostCsr C, S, K, B, Bt;
        std::vector<int> pord(std::max(rp, 1)), ppos(std::max(rp, 1));
        for (int r = 0; r < (int)pord.size(); ++r) pord[r] = ppos[r] = r;  // padding rows map to themselves
        for (int i = 0; i < ni; ++i) {
            // the potential rows in locality order: K's rows and columns, B's
            // output rows and B^T's columns; the multigrid hierarchy is built
            // on the free-node numbering and permuted when it is uploaded
            const std::vector<int> &ord = as[i].pot_order;
            std::vector<int> pos(np[i]);
            for (int r = 0; r < np[i]; ++r) {
                pos[ord[r]] = r;
                pord[poff[i] + r] = poff[i] + ord[r];
                ppos[poff[i] + ord[r]] = poff[i] + r;
            }
            c->inst[i].pot_order = ord;
            c->hostK.push_back(as[i].K);  // kept for the multigrid hierarchies
            as[i].K = permute_sym(as[i].K, ord, pos);
            for (int &o : as[i].B.row_out) o = pos[o];
            for (int &j : as[i].Bt.col) j = pos[j];
            to_difference_form(as[i].C);
            to_difference_form(as[i].S);
            append_csr(C, as[i].C, moff[i], moff[i], 0);
            append_csr(S, as[i].S, moff[i], moff[i], 0);
            append_csr(K, as[i].K, poff[i], poff[i], 0);
            append_csr(B, as[i].B, boff[i], moff[i], poff[i]);
            append_csr(Bt, as[i].Bt, moff[i], poff[i], 0);
            as[i].C = HostCsr();
            as[i].S = HostCsr();
            as[i].K = HostCsr();
            as[i].B = HostCsr();
            as[i].Bt = HostCsr();
        }
        pad_rows(C, rm);
        pad_rows(S, rm);
        pad_rows(K, rp);
        pad_rows(B, rb);
        pad_rows(Bt, rm);
        C.vw = 6;
        S.vw = 1;
        K.vw = 1;
        B.vw = 3;
        Bt.vw = 3;
        upload_sell(c, C, c->C);
        upload_sell(c, S, c->S);
        upload_sell(c, K, c->K);
        upload_sell(c, B, c->B);
        upload_sell(c, Bt, c->Bt);
        c->pord = dalloc_n<int>(c, pord.size());
        c->ppos = dalloc_n<int>(c, ppos.size());
        HIPCHK(hipMemcpyAsync(c->pord, pord.data(), pord.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->ppos, ppos.data(), ppos.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
        sync(c);
    }
    make_map(c, c->Mm, moff, nm, std::vector<int>(ni, kBlock / kSlice), true);
    make_map(c, c->Mb, boff, nb, std::vector<int>(ni, kBlock / kSlice), true);
    c->pnw = kPoissonWaves;
    c->pspw.assign(ni, 1);
    c->poff = poff;
    c->pn = np;
    make_map(c, c->Mp, poff, np, std::vector<int>(ni, kPoissonWaves));

    const size_t RM = std::max(rm, 1), RP = std::max(rp, 1);
    c->L = dalloc_n<double>(c, RM);
    c->invDex = dalloc_n<double>(c, RM);
    c->invDK = dalloc_n<double>(c, RP);
    c->invDK32 = dalloc_n<float>(c, RP);
    {
        std::vector<double> L(RM, 0.0), iD(RM, 1.0), iK(RP, 1.0);
        for (int i = 0; i < ni; ++i) {
            for (int a = 0; a < nm[i]; ++a) {
                L[moff[i] + a] = as[i].L[a];
                iD[moff[i] + a] = 1.0 / as[i].Dex[a];
            }
            for (int r = 0; r < np[i]; ++r) iK[poff[i] + r] = 1.0 / as[i].DK[c->inst[i].pot_order[r]];
        }
        upload_vec(c, c->L, L);
        upload_vec(c, c->invDex, iD);
        upload_vec(c, c->invDK, iK);
        launch_to_f32((int64_t)RP, c->invDK, c->invDK32, c->stream);
    }
    for (auto &s : c->st) {
        s.x = dalloc_n<double>(c, 3 * RM);
        s.G = dalloc_n<double>(c, 3 * RM);
        s.g = dalloc_n<double>(c, 3 * RM);
        s.lam = dalloc_n<double>(c, RM);
    }
    for (double **p : {&c->gprev, &c->d, &c->y, &c->pr, &c->pp, &c->pq, &c->tmp3}) *p = dalloc_n<double>(c, 3 * RM);
    c->dscale = dalloc_n<double>(c, RM);
    c->gy = dalloc_n<double>(c, 2 * (size_t)ni);
    HIPCHK(hipMemsetAsync(c->gy, 0, 2 * (size_t)ni * sizeof(double), c->stream));
    for (double **p : {&c->u, &c->b, &c->cr, &c->cq, &c->usave, &c->ux, &c->ut}) *p = dalloc_n<double>(c, RP);
    for (auto &q : c->q64) q = dalloc_n<PcgNode<double>>(c, RP);
    for (auto &q : c->q32) q = dalloc_n<PcgNode<float>>(c, RP);
    c->p64 = dalloc_n<double>(c, RP);
    c->p32 = dalloc_n<float>(c, RP);
    c->x32 = dalloc_n<float>(c, RP);
    c->pst = dalloc_n<PcgState>(c, ni);
    c->mpart = dalloc_n<double>(c, (size_t)MS_TOTAL * c->Mm.map.nblk);
    c->ppart = dalloc_n<double>(c, (size_t)kPcgSlots * c->Mp.map.nblk);
    // control block: 8 double arrays then 11 int arrays in one allocation, so
    // that one copy uploads the doubles and the first six int arrays; the
    // staged potential operations likewise: per slot, ninst doubles then
    // ninst ints
    const size_t ctl_bytes = 8 * (size_t)ni * sizeof(double) + 11 * (size_t)ni * sizeof(int);
    const size_t po_bytes = 2 * (size_t)ni * (sizeof(double) + sizeof(int));
    c->dcd = (double *)dalloc(c, ctl_bytes);
    c->dci = (int *)(c->dcd + 8 * (size_t)ni);
    c->dpr = (double *)dalloc(c, po_bytes);
    c->dsc = dalloc_n<double>(c, (size_t)SC_PER * ni);
    HIPCHK(hipHostMalloc((void **)&c->hcd, ctl_bytes, hipHostMallocDefault));
    c->hci = (int *)(c->hcd + 8 * (size_t)ni);
    HIPCHK(hipHostMalloc((void **)&c->hsc, (size_t)SC_PER * ni * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&c->hpst, (size_t)ni * sizeof(PcgState), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&c->hpr, po_bytes, hipHostMallocDefault));
    std::memset(c->hci, 0, 11 * (size_t)ni * sizeof(int));
    std::memset(c->hcd, 0, 8 * (size_t)ni * sizeof(double));
    std::memset(c->hsc, 0, (size_t)SC_PER * ni * sizeof(double));
    std::memset(c->hpst, 0, (size_t)ni * sizeof(PcgState));
    // every vector starts at zero (padding rows stay zero for good)
    for (const StateV &s : c->st) {
        HIPCHK(hipMemsetAsync(s.x, 0, 3 * RM * sizeof(double), c->stream));
        HIPCHK(hipMemsetAsync(s.G, 0, 3 * RM * sizeof(double), c->stream));
        HIPCHK(hipMemsetAsync(s.g, 0, 3 * RM * sizeof(double), c->stream));
        HIPCHK(hipMemsetAsync(s.lam, 0, RM * sizeof(double), c->stream));
    }
    for (double *p : {c->gprev, c->d, c->y, c->pr, c->pp, c->pq, c->tmp3})
        HIPCHK(hipMemsetAsync(p, 0, 3 * RM * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(c->dscale, 0, RM * sizeof(double), c->stream));
    for (double *p : {c->u, c->b, c->cr, c->cq, c->usave, c->ux, c->ut})
        HIPCHK(hipMemsetAsync(p, 0, RP * sizeof(double), c->stream));
    for (auto *q : c->q64) HIPCHK(hipMemsetAsync(q, 0, RP * sizeof(PcgNode<double>), c->stream));
    for (auto *q : c->q32) HIPCHK(hipMemsetAsync(q, 0, RP * sizeof(PcgNode<float>), c->stream));
    HIPCHK(hipMemsetAsync(c->p64, 0, RP * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(c->p32, 0, RP * sizeof(float), c->stream));
    HIPCHK(hipMemsetAsync(c->x32, 0, RP * sizeof(float), c->stream));
    HIPCHK(hipMemsetAsync(c->pst, 0, ni * sizeof(PcgState), c->stream));
    HIPCHK(hipMemsetAsync(c->mpart, 0, (size_t)MS_TOTAL * c->Mm.map.nblk * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(c->ppart, 0, (size_t)kPcgSlots * c->Mp.map.nblk * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(c->dci, 0, 11 * (size_t)ni * sizeof(int), c->stream));
    HIPCHK(hipMemsetAsync(c->dcd, 0, 8 * (size_t)ni * sizeof(double), c->stream));
    HIPCHK(hipMemsetAsync(c->dsc, 0, (size_t)SC_PER * ni * sizeof(double), c->stream));
    sync(c);
    c->last_pcg.assign((size_t)kPcgKinds * ni, 16);
    c->cnt.assign(ni, Cnt());
    c->pcg_bytes64.assign(ni, 0.0);
    c->pcg_bytes32.assign(ni, 0.0);
    for (int i = 0; i < ni; ++i) {
        // one iteration: the matrix (values + column indices) once; r, w, s,
        // D^-1, p, x read and r, w, s, p, x written once per row
        const double nnz = (double)c->inst[i].nnz_K, rows = (double)c->inst[i].n_pot;
        c->pcg_bytes64[i] = nnz * (8.0 + 4.0) + 11.0 * 8.0 * rows;
        c->pcg_bytes32[i] = nnz * (4.0 + 4.0) + 11.0 * 4.0 * rows;
    }
}

// ---------------------------------------------------------------------------
// scalar-potential solve K u = b (warm start u), Jacobi-PCG; FP64, or FP32 CG
// inside FP64 defect correction
// ---------------------------------------------------------------------------
PcgLaunch pcg_args(mm_ctx *c) {
    PcgLaunch a;
    a.K = &c->K;
    a.M = &c->Mp.map;
    a.st = c->pst;
    a.part = c->ppart;
    a.u = c->u;
    a.b = c->b;
    a.invD = c->invDK;
    a.r64 = c->cr;  // scratch: the FP64 residual of the defect correction
    a.v64 = PcgVecs<double>{{c->q64[0], c->q64[1]}, c->p64};
    a.x32 = c->x32;
    a.invD32 = c->invDK32;
    a.v32 = PcgVecs<float>{{c->q32[0], c->q32[1]}, c->p32};
    a.pin = c->d_(c->pin());
    a.nw = c->pnw;
    return a;
}

// kinds of scalar-potential CG: Jacobi (one kernel per iteration), multigrid
// in one precision, and multigrid in the mixed form of the FP32-bulk mode
enum CgKind { CG_JACOBI = 0, CG_AMG = 1, CG_AMG_MIXED = 2 };

void pcg_chunk(mm_ctx *c, bool fp32, int kind) {
    PcgLaunch a = pcg_args(c);
    if (kind != CG_JACOBI) {
        for (int j = 0; j < kAmgChunk; ++j) {
            if (kind == CG_AMG_MIXED)
                launch_amg_itermix(a, amg_launch32(c->amg), amg_launch64(c->amg), j & 1, c->stream);
            else launch_amg_iter64(a, amg_launch64(c->amg), j & 1, c->stream);
        }
        return;
    }
    for (int j = 0; j < kPcgChunk; ++j) {
        if (fp32) launch_pcg_iter32(a, j & 1, c->stream);
        else launch_pcg_iter64(a, j & 1, c->stream);
    }
}

bool use_graphs() {
    static bool on = [] {
        const char *e = std::getenv("MMNCG_NO_GRAPH");
        return !(e && std::atoi(e) != 0);
    }();
    return on;
}

// capture one chunk of iterations once per context, precision and
// preconditioner
hipGraphExec_t pcg_graph(mm_ctx *c, bool fp32, int kind) {
    hipGraphExec_t &ge = kind == CG_AMG_MIXED ? c->mgraph
                         : kind == CG_AMG    ? c->agraph64
                                             : (fp32 ? c->graph32 : c->graph64);
    if (ge) return ge;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    try {
        pcg_chunk(c, fp32, kind);
    } catch (...) {
        (void)hipStreamEndCapture(c->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    HIPCHK(hipStreamEndCapture(c->stream, &g));
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    return ge;
}

void pull_pcg(mm_ctx *c) {
    HIPCHK(hipMemcpyAsync(c->hpst, c->pst, c->ninst * sizeof(PcgState), hipMemcpyDeviceToHost, c->stream));
    sync(c);
}

// Replays graph chunks until every instance in `on` reports convergence;
// iteration counts are left in hpst. With timing on, HIP events bracket every
// batch of replays and the executed iterations (and their algorithmic bytes)
// are counted per instance; replays after an instance converged return at once
// and their time stays in the measurement.
// slot of last_pcg for instance i's current solve: the role of its evaluation
// (the accepted state, the line search's first or second trial: their starts
// differ in quality) and the defect-correction pass (the first pass does
// nearly all the work)
long &last_pcg_of(mm_ctx *c, int i) {
    const int rl = std::min(std::max(c->role()[i], 0), 2);
    return c->last_pcg[(size_t)kPcgKinds * i + 2 * rl + (c->pcg_pass > 0 ? 1 : 0)];
}

void pcg_replay(mm_ctx *c, bool fp32, int kind, long maxit, const std::vector<int> &on) {
    hipGraphExec_t ge = use_graphs() ? pcg_graph(c, fp32, kind) : nullptr;
    const long chunk = kind != CG_JACOBI ? kAmgChunk : kPcgChunk;
    long expect = chunk;
    for (int i : on) expect = std::max(expect, last_pcg_of(c, i));
    long nrep = (expect + chunk - 1) / chunk;
    long launched = 0;
    std::vector<int> seen(c->ninst, 0);
    std::vector<double> bytes = fp32 ? c->pcg_bytes32 : c->pcg_bytes64;
    if (kind != CG_JACOBI) bytes = amg_bytes(c->amg, kind == CG_AMG_MIXED ? 2 : 0);
    for (;;) {
        prof_mark(c);
        for (long k = 0; k < nrep; ++k) {
            if (ge) HIPCHK(hipGraphLaunch(ge, c->stream));
            else pcg_chunk(c, fp32, kind);
        }
        prof_mark(c);
        launched += nrep * chunk;
        pull_pcg(c);
        if (c->prof_on) {
            prof_harvest(c);
            for (int i : on) {
                int di = c->hpst[i].iters - seen[i];
                c->prof_units += di;
                c->prof_bytes += di * bytes[i];
                seen[i] = c->hpst[i].iters;
            }
        }
        bool all = true;
        for (int i : on) all = all && (c->hpst[i].done || c->hpst[i].zero_u);
        if (all) break;
        if (launched >= maxit) throw ApiError{MM_NOT_CONVERGED, "scalar-potential CG did not converge"};
        nrep = std::max<long>(1, (expect / 8 + chunk - 1) / chunk);
    }
}

void zero_pot(mm_ctx *c, int i) {
    launch_fill(c->inst[i].n_pot, c->u + c->inst[i].pot_off, 0.0, c->stream);
}

// FP64 CG for the instances with act[i] set (uploaded); returns per-instance iterations
// FP64 CG vectors and residual norms: the FP64 mode (Jacobi or multigrid),
// and the mixed multigrid form of the FP32-bulk mode (FP32-stored matrix and
// cycle), which needs no defect correction
std::vector<long> poisson_fp64(mm_ctx *c, double rtol, long maxit, int kind, const std::vector<int> &on) {
    std::vector<long> it(c->ninst, 0);
    PcgLaunch a = pcg_args(c);
    const int *act = c->d_(c->act());
    if (kind == CG_AMG_MIXED)
        launch_amg_initmix(a, amg_launch32(c->amg), amg_launch64(c->amg), act, rtol * rtol, c->stream);
    else if (kind == CG_AMG) launch_amg_init64(a, amg_launch64(c->amg), act, rtol * rtol, c->stream);
    else launch_pcg_init64(a, act, rtol * rtol, c->stream);
    pcg_replay(c, false, kind, maxit, on);
    for (int i : on) {
        if (c->hpst[i].zero_u) {
            zero_pot(c, i);
            continue;
        }
        it[i] = c->hpst[i].iters;
        last_pcg_of(c, i) = std::max<long>(4, it[i]);
    }
    return it;
}

std::vector<long> poisson_fp32(mm_ctx *c, double rtol, long maxit, const std::vector<int> &on) {
    std::vector<long> total(c->ninst, 0);
    PcgLaunch a = pcg_args(c);
    std::vector<int> live = on;
    int *pl = c->plive();
    double *pin = c->pin();
    for (int outer = 0; outer < 50 && !live.empty(); ++outer) {
        // the first residual serves the instances of act[] (already uploaded);
        // later ones the instances still correcting (the host writes plive
        // only after the synchronization of the previous pass)
        const int *live_dev = c->d_(c->act());
        if (outer > 0) {
            std::fill(pl, pl + c->ninst, 0);
            for (int i : live) pl[i] = 1;
            upload_ctl(c);
            live_dev = c->d_(pl);
        }
        launch_residual64(a, live_dev, c->stream);
        pull_pcg(c);
        std::vector<int> inner;
        for (int k = 0; k < c->ninst; ++k) pin[4 * k + 1] = 0.0;
        for (int i : live) {
            const double bb = c->hpst[i].bb, rr = c->hpst[i].rr;
            if (bb == 0.0) {
                zero_pot(c, i);
                continue;
            }
            if (rr <= rtol * rtol * bb) continue;
            const double rn = std::sqrt(rr);
            // relative target of the inner FP32 solve: what the outer FP64 test
            // needs and no more (the CG stops below it; a pass that ends short
            // is followed by one more), floored at 1e-5 where FP32 runs out
            double tol = std::max(1e-5, rtol * std::sqrt(bb) / rn);
            tol = std::min(tol, 1e-1);
            pin[4 * i] = 1.0 / rn;
            pin[4 * i + 1] = tol * tol;
            pin[4 * i + 2] = rn;
            inner.push_back(i);
        }
        live = inner;
        if (live.empty()) break;
        upload_ctl(c);
        launch_pcg_init32(a, c->stream);
        long cap = 0;
        for (int i : live) cap = std::max(cap, maxit - total[i]);
        c->pcg_pass = outer;
        pcg_replay(c, true, CG_JACOBI, cap, live);
        for (int i : live) {
            total[i] += c->hpst[i].iters;
            last_pcg_of(c, i) = std::max<long>(4, c->hpst[i].iters);
            if (total[i] >= maxit) throw ApiError{MM_NOT_CONVERGED, "scalar-potential CG did not converge"};
        }
        launch_add_correction(a, c->stream);
    }
    c->pcg_pass = 0;
    if (!live.empty()) throw ApiError{MM_NOT_CONVERGED, "scalar-potential defect correction did not converge"};
    for (int k = 0; k < c->ninst; ++k) pin[4 * k + 1] = 0.0;
    return total;
}

// solve for the instances in `on` (act[] uploaded with exactly these set)
void poisson(mm_ctx *c, double rtol, long maxit, bool fp32, bool amg, const std::vector<int> &on) {
    if (on.empty() || c->rows_p == 0) return;
    c->pcg_pass = 0;
    if (amg) amg_get(c);  // first use: build the hierarchy (untimed, like the assembly)
    const double t0 = now_s();
    std::vector<long> it = (fp32 && amg)  ? poisson_fp64(c, rtol, maxit, CG_AMG_MIXED, on)
                           : fp32         ? poisson_fp32(c, rtol, maxit, on)
                                          : poisson_fp64(c, rtol, maxit, amg ? CG_AMG : CG_JACOBI, on);
    sync(c);
    const double dt = now_s() - t0;
    for (int i : on) {
        c->cnt[i].mi += it[i];
        c->cnt[i].t_mag += dt;
    }
}

// ---------------------------------------------------------------------------
// block shape of the scalar-potential kernels and its autotuner
// ---------------------------------------------------------------------------
// Rebuilds the potential-row map for nw waves per block and spw[i] slices per
// wave of instance i. Captured graphs hold the old map: they are dropped.
void set_poisson_shape(mm_ctx *c, int nw, const std::vector<int> &spw, int bm = 1) {
    sync(c);
    for (hipGraphExec_t *g : {&c->graph64, &c->graph32, &c->agraph64, &c->mgraph}) {
        if (*g) (void)hipGraphExecDestroy(*g);
        *g = nullptr;
    }
    dfree(c, (void *)c->Mp.map.tab);
    dfree(c, (void *)c->Mp.map.ipb);
    dfree(c, (void *)c->Mp.map.rend);
    std::vector<int> spb(c->ninst);
    for (int i = 0; i < c->ninst; ++i) spb[i] = nw * spw[i];
    const int old = c->Mp.map.nblk;
    make_map(c, c->Mp, c->poff, c->pn, spb, false, bm);
    if (c->Mp.map.nblk > old) {
        dfree(c, c->ppart);
        c->ppart = dalloc_n<double>(c, (size_t)kPcgSlots * c->Mp.map.nblk);
        HIPCHK(hipMemsetAsync(c->ppart, 0, (size_t)kPcgSlots * c->Mp.map.nblk * sizeof(double), c->stream));
        sync(c);
    }
    c->pnw = nw;
    c->pspw = spw;
    c->pbm = bm;
}

// size bucket of an instance for the tuner: floor(log2(n_pot / 4096)), 0..7
int size_bucket(int n_pot) {
    int b = 0;
    for (long v = n_pot / 4096; v > 1 && b < 7; v >>= 1) ++b;
    return b;
}

// Average time of one CG iteration (seconds) over the instances in `on`, for
// the current block shape: a synthetic right-hand side (b = 1 on every free
// node, u = 0), a tolerance that never stops, 4 untimed and 32 timed eager
// iterations, best of 3. The caller saves and restores u and b.
double time_pcg(mm_ctx *c, const std::vector<int> &on, bool fp32) {
    hipStream_t s = c->stream;
    PcgLaunch a = pcg_args(c);
    std::fill(c->act(), c->act() + c->ninst, 0);
    for (int k = 0; k < c->ninst; ++k) c->pin()[4 * k + 1] = 0.0;
    for (int i : on) {
        c->act()[i] = 1;
        c->pin()[4 * i] = 1.0;
        c->pin()[4 * i + 1] = 1e-300;
        c->pin()[4 * i + 2] = 1.0;
    }
    upload_ctl(c);
    double best = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
        launch_fill(c->rows_p, c->b, 1.0, s);
        launch_fill(c->rows_p, c->u, 0.0, s);
        if (fp32) {
            // the FP32 inner solve starts from the FP64 residual, as in the defect correction
            launch_residual64(a, c->d_(c->act()), s);
            launch_pcg_init32(a, s);
        } else {
            launch_pcg_init64(a, c->d_(c->act()), 0.0, s);
        }
        for (int j = 0; j < 4; ++j) fp32 ? launch_pcg_iter32(a, j & 1, s) : launch_pcg_iter64(a, j & 1, s);
        HIPCHK(hipEventRecord(c->ev[0], s));
        for (int j = 0; j < 32; ++j) fp32 ? launch_pcg_iter32(a, j & 1, s) : launch_pcg_iter64(a, j & 1, s);
        HIPCHK(hipEventRecord(c->ev[1], s));
        HIPCHK(hipEventSynchronize(c->ev[1]));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        best = std::min(best, ms * 1e-3 / 32.0);
    }
    sync(c);
    std::fill(c->act(), c->act() + c->ninst, 0);
    for (int k = 0; k < c->ninst; ++k) c->pin()[4 * k + 1] = 0.0;
    return best;
}

// One cached result: the shape chosen for a batch of this composition
// (`batch` lists the size buckets present with their instance counts; `spw`
// the slices per wave of those buckets in the same order) and its measured
// time per CG iteration of the whole batch.
struct TuneEntry {
    std::string device, batch, spw;
    int fp32, nw, bm;
    double us;
};

std::string device_key(mm_ctx *c) {
    hipDeviceProp_t p;
    HIPCHK(hipGetDeviceProperties(&p, c->device));
    // architecture and compute units only: the marketing name is not stable
    // (a profiler's runtime reports another one)
    std::string k = std::string(p.gcnArchName) + ":cu" + std::to_string(p.multiProcessorCount);
    for (char &ch : k)
        if (ch == '"' || ch == '\\' || ch == '\n') ch = '_';
    return k;
}

// the cache is JSON with one entry object per line (written by tune_write)
std::vector<TuneEntry> tune_read(const char *path) {
    std::vector<TuneEntry> out;
    if (!path) return out;
    FILE *f = std::fopen(path, "r");
    if (!f) return out;
    char line[2048];
    while (std::fgets(line, sizeof line, f)) {
        char dev[512], batch[512], spw[512];
        TuneEntry e;
        if (std::sscanf(line,
                        " {\"device\": \"%511[^\"]\", \"fp32\": %d, \"batch\": \"%511[^\"]\", \"nw\": %d, "
                        "\"bm\": %d, \"spw\": \"%511[^\"]\", \"us\": %lf}",
                        dev, &e.fp32, batch, &e.nw, &e.bm, spw, &e.us) == 7) {
            e.device = dev;
            e.batch = batch;
            e.spw = spw;
            out.push_back(e);
        }
    }
    std::fclose(f);
    return out;
}
void tune_write(const char *path, const std::vector<TuneEntry> &v) {
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) throw ApiError{MM_EINVAL, std::string("cannot write tuning cache ") + path};
    std::fprintf(f, "{\"mmncg_tune\": 3, \"entries\": [\n");
    for (size_t k = 0; k < v.size(); ++k)
        std::fprintf(f,
                     "  {\"device\": \"%s\", \"fp32\": %d, \"batch\": \"%s\", \"nw\": %d, \"bm\": %d, "
                     "\"spw\": \"%s\", \"us\": %.4f}%s\n",
                     v[k].device.c_str(), v[k].fp32, v[k].batch.c_str(), v[k].nw, v[k].bm, v[k].spw.c_str(), v[k].us,
                     k + 1 < v.size() ? "," : "");
    std::fprintf(f, "]}\n");
    std::fclose(f);
    if (std::rename(tmp.c_str(), path) != 0) throw ApiError{MM_EINVAL, std::string("cannot write ") + path};
}

constexpr int kTuneNw[3] = {4, 8, 16};
constexpr int kTuneSpw[3] = {1, 2, 4};
constexpr int kTuneBm[3] = {1, 2, 4};  // multipliers of the blocks-per-instance cap

// Picks the block shape by timing CG iterations of the whole batch (every
// instance active, synthetic right-hand side): for every waves-per-block
// value, first one slices-per-wave value for all size buckets, then each
// bucket's value in turn with the others fixed; the fastest waves-per-block
// value wins. With a cache, a batch of the same composition on the same
// device and precision reuses the stored choice without timing.
void autotune(mm_ctx *c, bool use_cache, const char *path, bool fp32) {
    const int ni = c->ninst;
    std::vector<int> bucket(ni);
    std::vector<std::vector<int>> members(8);
    std::vector<int> all;
    for (int i = 0; i < ni; ++i) {
        bucket[i] = size_bucket(c->pn[i]);
        if (c->pn[i] > 0) {
            members[bucket[i]].push_back(i);
            all.push_back(i);
        }
    }
    std::vector<int> present;
    std::string sig;
    for (int b = 0; b < 8; ++b)
        if (!members[b].empty()) {
            present.push_back(b);
            sig += (sig.empty() ? "" : "+") + std::string("b") + std::to_string(b) + "x" +
                   std::to_string(members[b].size());
        }
    const std::string dev = device_key(c);
    std::vector<TuneEntry> cache = use_cache ? tune_read(path) : std::vector<TuneEntry>();
    auto apply = [&](int nw, const std::vector<int> &bspw, int bm) {
        std::vector<int> spw(ni, 1);
        for (size_t k = 0; k < present.size(); ++k)
            for (int i : members[present[k]]) spw[i] = bspw[k];
        set_poisson_shape(c, nw, spw, bm);
    };
    for (const TuneEntry &e : cache) {
        if (e.device != dev || e.fp32 != (fp32 ? 1 : 0) || e.batch != sig) continue;
        std::vector<int> bspw;
        size_t pos = 0;
        while (pos <= e.spw.size() && bspw.size() < present.size()) {
            bspw.push_back(std::atoi(e.spw.c_str() + pos));
            size_t nx = e.spw.find(',', pos);
            if (nx == std::string::npos) break;
            pos = nx + 1;
        }
        bool ok = bspw.size() == present.size() && (e.nw == 4 || e.nw == 8 || e.nw == 16) &&
                  (e.bm == 1 || e.bm == 2 || e.bm == 4);
        for (int v : bspw) ok = ok && (v == 1 || v == 2 || v == 4);
        if (!ok) continue;
        apply(e.nw, bspw, e.bm);
        c->tuned = true;
        return;
    }
    // keep the warm start and the right-hand side aside
    const size_t RP = std::max(c->rows_p, 1);
    HIPCHK(hipMemcpyAsync(c->usave, c->u, RP * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    double best_t = 1e300;
    int best_nw = kPoissonWaves, best_bm = 1;
    std::vector<int> best_b(present.size(), 1);
    for (int bm : kTuneBm)
        for (int nw : kTuneNw) {
            std::vector<int> bspw(present.size(), 1);
            double tcur = 1e300;
            for (int cand : kTuneSpw) {
                std::vector<int> trial(present.size(), cand);
                apply(nw, trial, bm);
                const double t = time_pcg(c, all, fp32);
                if (t < tcur) {
                    tcur = t;
                    bspw = trial;
                }
            }
            if (present.size() > 1)
                for (size_t k = 0; k < present.size(); ++k)
                    for (int cand : kTuneSpw) {
                        if (cand == bspw[k]) continue;
                        std::vector<int> trial = bspw;
                        trial[k] = cand;
                        apply(nw, trial, bm);
                        const double t = time_pcg(c, all, fp32);
                        if (t < tcur) {
                            tcur = t;
                            bspw = trial;
                        }
                    }
            if (tcur < best_t) {
                best_t = tcur;
                best_nw = nw;
                best_b = bspw;
                best_bm = bm;
            }
        }
    apply(best_nw, best_b, best_bm);
    launch_fill((int64_t)RP, c->b, 0.0, c->stream);
    HIPCHK(hipMemcpyAsync(c->u, c->usave, RP * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    upload_ctl(c);
    sync(c);
    if (use_cache) {
        std::string spw;
        for (size_t k = 0; k < best_b.size(); ++k) spw += (k ? "," : "") + std::to_string(best_b[k]);
        cache.push_back(TuneEntry{dev, sig, spw, fp32 ? 1 : 0, best_nw, best_bm, best_t * 1e6});
        tune_write(path, cache);
    }
    c->tuned = true;
}

// ---------------------------------------------------------------------------
// batched evaluation: every instance with act[i] evaluates its state role[i]
// (0 current; 1, 2: trial N(x + alpha_i d) relative to the current state).
// Fills act/role/alpha/h3 of the control block beforehand.
// ---------------------------------------------------------------------------
int cmode_of(int terms) { return ((terms & MM_T_EXCH) ? 1 : 0) | ((terms & MM_T_ANIS) ? 2 : 0); }

// Algorithmic bytes of the timed field kernels over the instances in `on`:
// each stored operator entry (values and column index) once, each magnet-node
// vector the kernel reads or writes once. v is the operator value size.
double eval_bytes(mm_ctx *c, const mm_opts &o, const std::vector<int> &on, bool demag, double v) {
    const int cm = cmode_of(o.terms);
    double b = 0;
    for (int i : on) {
        const InstInfo &I = c->inst[i];
        if (cm & 2) b += I.nnz_C * (6 * v + 4);
        if (cm == 1 || cm == 2) b += I.nnz_S * (v + 4);
        if (demag) b += I.nnz_B * (3 * v + 4);  // B^T holds B's entries
        // m (24), L (8) read; G (24), g (24), lambda (8) written; a line-search
        // trial also reads x0 (24), d (24), g0 (24), lambda0 (8)
        b += I.n_mag * (88.0 + (c->role()[i] != 0 ? 80.0 : 0.0));
    }
    return b;
}
double bmul_bytes(mm_ctx *c, const std::vector<int> &on, double v) {
    double b = 0;
    for (int i : on) {
        const InstInfo &I = c->inst[i];
        b += I.nnz_B * (3 * v + 4) + 24.0 * I.n_mag + 8.0 * I.n_brow;  // B, m read, b written
    }
    return b;
}
double prec_apply_bytes(mm_ctx *c, int form, double v) {
    double b = 0;
    for (int i = 0; i < c->ninst; ++i) {
        if (!c->pact()[i]) continue;
        const InstInfo &I = c->inst[i];
        // C, then m (24), lambda (8), p (24) read and q (24) written (+ g with all four terms)
        b += I.nnz_C * (6 * v + 4) + I.n_mag * (80.0 + (form == MM_PFORM_FULL ? 24.0 : 0.0));
    }
    return b;
}

void eval_round(mm_ctx *c, const mm_opts &o, const std::vector<int> &on, bool any_trial) {
    hipStream_t s = c->stream;
    const bool fp32 = o.precision == MM_FP32_BULK;
    if (!(o.terms & MM_T_ZEE)) std::fill(c->h3(), c->h3() + 3 * c->ninst, 0.0);
    upload_ctl(c);
    const int *act = c->d_(c->act()), *role = c->d_(c->role());
    const double *alpha = c->d_(c->alpha());
    if (any_trial) launch_trial(c->Mm.map, act, role, c->st, c->d, alpha, s);
    const bool demag = (o.terms & MM_T_DEMAG) && c->rows_p > 0 && c->B.nrows > 0;
    const double v = fp32 ? 4.0 : 8.0;
    if (demag) {
        kt_begin(c, KT_BMUL);
        launch_bmul(c->B, c->Mb.map, act, c->st, role, c->b, fp32, s);
        if (c->kt_on) kt_end(c, KT_BMUL, bmul_bytes(c, on, v));
        poisson(c, o.poisson_rtol, o.poisson_maxit, fp32, o.poisson_prec == MM_PREC_AMG, on);
    }
    EvalLaunch e;
    e.C = &c->C;
    e.S = &c->S;
    e.Bt = &c->Bt;
    e.M = &c->Mm.map;
    e.cmode = cmode_of(o.terms);
    e.use_demag = demag ? 1 : 0;
    e.act = act;
    e.role = role;
    for (int k = 0; k < 3; ++k) e.st[k] = c->st[k];
    e.u = c->u;
    e.L = c->L;
    e.h3 = c->d_(c->h3());
    e.d = c->d;
    e.alpha = alpha;
    e.part = mslot(c, MS_EVAL);
    e.fp32 = fp32;
    kt_begin(c, KT_EVAL);
    launch_eval_epilogue(e, s);
    if (c->kt_on) kt_end(c, KT_EVAL, eval_bytes(c, o, on, demag, v));
    launch_finalize_inst(c->Mm.map, mslot(c, MS_EVAL), kEvalParts, eval_max_mask(), dsc_at(c, SC_EVAL), s);
    pull_sc(c, SC_EVAL, kEvalParts);
    sync(c);
    for (int i : on) c->cnt[i].evals++;
}

Sc eval_result(mm_ctx *c, int i) {
    const double *r = hsc_at(c, SC_EVAL) + (size_t)kEvalParts * i;
    Sc v;
    v.Eloc = r[0];
    v.Ez = r[1];
    v.Ed = r[2];
    v.E = r[0] + r[1] + r[2];
    v.dF = r[3];
    v.dphi = r[4];
    v.tmax = r[6];
    v.ginf = r[7];
    v.dxinf = r[8];
    v.minf = r[9];
    return v;
}

// exchange / anisotropy split of Eloc for instance i at the current state
void energy_parts(mm_ctx *c, int i, const Sc &v, const mm_opts &o, double E[5]) {
    const bool fp32 = o.precision == MM_FP32_BULK;
    double ex = 0.0, an = 0.0;
    const int cm = cmode_of(o.terms);
    if (cm == 3) {
        launch_energy_split(c->S, c->Mm.map, c->st[0].x, mslot(c, MS_MISC), fp32, c->stream);
        launch_finalize_inst(c->Mm.map, mslot(c, MS_MISC), 1, 0u, dsc_at(c, SC_MISC), c->stream);
        pull_sc(c, SC_MISC, 1);
        sync(c);
        ex = hsc_at(c, SC_MISC)[i];
        an = v.Eloc - ex;
    } else if (cm == 1) {
        ex = v.Eloc;
    } else if (cm == 2) {
        an = v.Eloc;
    }
    E[0] = ex;
    E[1] = an;
    E[2] = v.Ez;
    E[3] = v.Ed;
    E[4] = v.E;
}

// preconditioner for the instances with pact[i]: at most jmax steps of Alg. 1
// on P y = g at the current state (exits li1-li3)
// the exit flags of the inner solve, device -> host (pflags of the control block)
void pull_prec_flags(mm_ctx *c, const int *dflags) {
    if (dflags == c->d_(c->pflags())) return pull_flags(c);
    HIPCHK(hipMemcpyAsync(c->pflags(), dflags, 4 * (size_t)c->ninst * sizeof(int), hipMemcpyDeviceToHost,
                          c->stream));
}

size_t prec_scratch_bytes(const mm_ctx *c) {
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t v3 = al(3 * (size_t)std::max(c->rows_m, 1) * sizeof(double));
    return 3 * v3 + al(7 * (size_t)c->Mm.map.nblk * sizeof(double)) + al(4 * (size_t)c->ninst * sizeof(int));
}
PrecScratch prec_scratch_at(const mm_ctx *c, void *base) {
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t v3 = al(3 * (size_t)std::max(c->rows_m, 1) * sizeof(double));
    char *b = (char *)base;
    PrecScratch s;
    s.r = (double *)b;
    s.p = (double *)(b + v3);
    s.q = (double *)(b + 2 * v3);
    s.part = (double *)(b + 3 * v3);
    s.flags = (int *)(b + 3 * v3 + al(7 * (size_t)c->Mm.map.nblk * sizeof(double)));
    return s;
}

void precondition(mm_ctx *c, int jmax, const double *dscale, bool fp32, int form, const PrecScratch *ext = nullptr) {
    PrecLaunch a;
    a.C = &c->C;
    a.M = &c->Mm.map;
    a.act = c->d_(c->pact());
    a.m = c->st[0].x;
    a.lam = c->st[0].lam;
    a.g = c->st[0].g;
    a.invDex = c->invDex;
    a.dscale = dscale;
    a.y = c->y;
    a.r = ext ? ext->r : c->pr;
    a.p = ext ? ext->p : c->pp;
    a.q = ext ? ext->q : c->pq;
    a.part = ext ? ext->part : mslot(c, MS_PREC);
    a.flags = ext ? ext->flags : c->d_(c->pflags());
    a.fp32 = fp32;
    a.form = form;
    launch_prec_init(a, c->stream);
    // An instance that has left by (li2) or (li3) makes the later launches
    // return at once, but each still costs a launch. Past kPrecCheck
    // iterations the host reads the exit flags every kPrecCheck iterations
    // and stops launching once every instance has left; below that no host
    // round trip is added.
    for (int j = 0; j < jmax; ++j) {
        // the first application always works on every active instance: it is
        // the one timed (later ones may return at once after an exit)
        if (j == 0) kt_begin(c, KT_PREC_APPLY);
        launch_prec_apply(a, j, c->stream);
        if (j == 0 && c->kt_on) kt_end(c, KT_PREC_APPLY, prec_apply_bytes(c, form, fp32 ? 4.0 : 8.0));
        launch_prec_tail(a, j, j + 1 == jmax, c->stream);
        if ((j + 1) % kPrecCheck == 0 && j + 1 < jmax) {
            pull_prec_flags(c, a.flags);
            sync(c);
            bool running = false;
            for (int i = 0; i < c->ninst && !running; ++i)
                running = c->pact()[i] && c->pflags()[4 * i] == 0;
            if (!running) break;
        }
    }
}

// load m (caller layout, host or device) into the current state and check
// that it holds finite unit vectors
void load_m(mm_ctx *c, const double *m) {
    for (const InstInfo &I : c->inst)
        copy_in(c, c->st[0].x + 3 * (size_t)I.mag_off, m + 3 * I.user_off, 3 * (size_t)I.n_mag);
    launch_mavg(c->Mm.map, c->st[0].x, c->L, mslot(c, MS_MISC), c->stream);
    launch_finalize_inst(c->Mm.map, mslot(c, MS_MISC), 5, 1u << 4, dsc_at(c, SC_MISC), c->stream);
    pull_sc(c, SC_MISC, 5);
    sync(c);
    for (int i = 0; i < c->ninst; ++i) {
        double dev = hsc_at(c, SC_MISC)[5 * i + 4];
        if (!(dev <= 1e-6))
            throw ApiError{MM_EINVAL, "m must hold finite unit vectors (instance " + std::to_string(i) +
                                          ": max | |m_i| - 1 | = " + std::to_string(dev) + ")"};
    }
}
void store_m(mm_ctx *c, double *m) {
    for (const InstInfo &I : c->inst)
        copy_out(c, m + 3 * I.user_off, c->st[0].x + 3 * (size_t)I.mag_off, 3 * (size_t)I.n_mag);
}

void reduce_field(const InstInfo &I, const double *BT, double h[3]) {
    for (int k = 0; k < 3; ++k) h[k] = BT[k] / (kMu0 * I.Ms_ref);
}

void set_h3(mm_ctx *c, int i, const double h[3]) {
    for (int k = 0; k < 3; ++k) c->h3()[3 * i + k] = h[k];
}

// ---------------------------------------------------------------------------
// the batched minimizer: Alg. 4 per instance over its list of field values
// ---------------------------------------------------------------------------
// Interpolation step of the line search: phi(a) = dp0 a + q a^2 + k a^3 is the
// cubic with phi(0) = 0, phi'(0) = dp0 that also meets phi(at) = dFt and
// phi'(at) = dpt. Its local minimizer is the root of phi'(a) = dp0 + 2 q a +
// 3 k a^2 where phi'' = 2 sqrt(q^2 - 3 k dp0) > 0, written without the
// cancellation of the textbook root: a = -dp0 / (q + sqrt(q^2 - 3 k dp0)).
// k = 0 (a parabola) needs no special case. No local minimizer: false.
bool cubic_step(double at, double dFt, double dp0, double dpt, double *ac) {
    const double slope = dFt / at;                        // secant slope over [0, at]
    const double k = (dp0 + dpt - 2.0 * slope) / (at * at);
    const double q = (3.0 * slope - 2.0 * dp0 - dpt) / at;
    const double disc = q * q - 3.0 * k * dp0;
    if (!(disc >= 0.0) || !std::isfinite(disc)) return false;
    const double den = q + std::sqrt(disc);
    if (!(den > 0.0) || !std::isfinite(den)) return false;
    const double a = -dp0 / den;
    if (!std::isfinite(a)) return false;
    *ac = a;
    return true;
}

int trace_level() {
    static int lvl = [] {
        const char *e = std::getenv("MMNCG_TRACE");
        return e ? std::atoi(e) : 0;
    }();
    return lvl;
}

enum Step { S_IDLE = 0, S_EVAL0, S_LEARN_T, S_TRIAL_T, S_TRIAL_C, S_HALVE, S_NEED_DIR, S_FIELD_DONE };

struct Run {
    int step = S_IDLE;
    long field = 0;
    double h[3] = {0, 0, 0};
    Sc cur, trial;
    // direction state
    int dirmode = 0;         // first[] bits for the next direction
    bool restarting = false;  // the next direction is the steepest-descent restart
    bool first = true;
    double dp0 = 0, dmax = 0, a_prev = 0, dp_prev = 0;
    double theta = 0;        // the line search's rotation cap of this field
    // line search
    bool restart_ls = false, arm_t = false;
    double amax = 0, a0 = 0, at = 0, ac = 0, a = 0, dFt = 0;
    Sc sT;                   // scalars of the trial kept in buffer T
    int halvings = 0;
    // per-field accounting
    long nli = 0, restarts = 0, fallbacks = 0;
    Cnt c0;
    double t0 = 0;
    int status = MM_OK;
    bool prec_ran = false;
    bool scaled = false;     // the learned Jacobi factors apply to this field
};

struct CurveOut {
    double *m_avg = nullptr;    // [ninst][nfield][3]
    double *E_tot = nullptr;    // [ninst][nfield]
    mm_stats *st = nullptr;     // [ninst][nfield]
    double *m_hist = nullptr;   // single instance: [nfield][n_mag][3]
    int *accepted = nullptr;    // single instance, learned start: [nfield] 1 when taken
};

// learned warm start / scaling (single instance): bits of `mode`
struct Learned {
    mm_gnn *net = nullptr;
    mm_graph *graph = nullptr;
    int mode = 0;
    bool has_prev = false;        // the curve continues from a minimizer at h_prev
    double h_prev[3] = {0, 0, 0};  // reduced units
};

// Per-instance operations on the scalar potential (launch_pot_op) staged in
// slot `slot` (0 before an evaluation round, 1 after it) of the pinned
// arrays: the driver synchronizes at least once between two uses of a slot.
void pot_ops(mm_ctx *c, int slot, const std::vector<int> &op, const std::vector<double> &rho) {
    const int n = c->ninst;
    bool any = false;
    for (int i = 0; i < n; ++i) any = any || op[i] != POT_NONE;
    if (!any) return;
    // slot layout: n doubles (rho), then n ints (op); one copy per call
    const size_t stride = (size_t)n * (sizeof(double) + sizeof(int));
    char *hb = (char *)c->hpr + slot * stride, *db = (char *)c->dpr + slot * stride;
    double *hr = (double *)hb;
    int *ho = (int *)(hb + (size_t)n * sizeof(double));
    for (int i = 0; i < n; ++i) {
        hr[i] = rho[i];
        ho[i] = op[i];
    }
    HIPCHK(hipMemcpyAsync(db, hb, stride, hipMemcpyHostToDevice, c->stream));
    launch_pot_op(c->Mp.map, (const int *)(db + (size_t)n * sizeof(double)), (const double *)db, c->u, c->ux, c->ut,
                  c->stream);
}

class Driver {
public:
    Driver(mm_ctx *c, const mm_opts &o, const std::vector<double> &hred, long nfield, const CurveOut &out,
           Learned ln = Learned())
        : c_(c), o_(o), h_(hred), nf_(nfield), out_(out), r_(c->ninst), ln_(ln) {}

    int run() {
        const int n = c_->ninst;
        for (int i = 0; i < n; ++i) start_field(i, 0);
        for (;;) {
            // ---- 1. evaluation of every instance that needs one
            std::vector<int> on;
            bool any_trial = false;
            for (int i = 0; i < n; ++i) {
                Run &R = r_[i];
                int a = 0, rl = 0;
                double al = 0.0;
                switch (R.step) {
                    case S_EVAL0: a = 1; break;
                    case S_LEARN_T: a = 1; rl = 1; al = 1.0; break;
                    case S_TRIAL_T: a = 1; rl = 1; al = R.at; break;
                    case S_HALVE: a = 1; rl = 1; al = R.a; break;
                    case S_TRIAL_C: a = 1; rl = 2; al = R.ac; break;
                    default: break;
                }
                c_->act()[i] = a;
                c_->role()[i] = rl;
                c_->alpha()[i] = al;
                c_->from()[i] = 0;
                c_->pact()[i] = 0;
                c_->first()[i] = 0;
                set_h3(c_, i, R.h);
                if (a) on.push_back(i);
                any_trial = any_trial || rl != 0;
            }
            bool busy = !on.empty();
            for (int i = 0; i < n; ++i) busy = busy || r_[i].step == S_NEED_DIR || r_[i].step == S_FIELD_DONE;
            if (!busy) break;
            if (!on.empty()) {
                // the scalar potential's start: a trial of role 2 (the line
                // search's second point on the same direction) starts from the
                // potentials at the accepted state and at the first trial,
                // interpolated linearly in alpha (the potential is linear in m,
                // and N(x + alpha d) departs from the line by O(alpha^2));
                // every other evaluation starts from the last potential
                std::vector<int> op(n, POT_NONE);
                std::vector<double> rho(n, 0.0);
                for (int i : on)
                    if (r_[i].step == S_TRIAL_C && r_[i].at > 0.0) {
                        op[i] = POT_INTERP;
                        rho[i] = r_[i].ac / r_[i].at;
                    }
                pot_ops(c_, 0, op, rho);
                std::vector<int> role_of(n, 0);
                for (int i : on) role_of[i] = c_->role()[i];
                eval_round(c_, o_, on, any_trial);
                for (int i : on) after_eval(i, eval_result(c_, i));
                // keep the potentials of the accepted state (ux) and of the
                // last role-1 trial (ut)
                std::fill(op.begin(), op.end(), POT_NONE);
                for (int i : on) {
                    const int from = c_->from()[i];
                    if (role_of[i] == 0) op[i] = POT_UX_U;
                    else if (role_of[i] == 1) op[i] = from == 1 ? POT_BOTH_U : POT_UT_U;
                    else op[i] = from == 2 ? POT_UX_U : (from == 1 ? POT_UX_UT : POT_NONE);
                }
                pot_ops(c_, 1, op, rho);
            }
            // ---- 2. copy accepted trials, precondition and direction
            std::vector<int> dir, fin;
            bool any_from = false, any_prec = false;
            for (int i = 0; i < n; ++i) {
                Run &R = r_[i];
                c_->act()[i] = 0;
                any_from = any_from || c_->from()[i] != 0;
                if (R.step == S_NEED_DIR) {
                    c_->act()[i] = 1;
                    c_->first()[i] = R.dirmode;
                    R.prec_ran = !(R.dirmode & 2) && o_.jmax > 0;
                    c_->pact()[i] = R.prec_ran ? 1 : 0;
                    any_prec = any_prec || R.prec_ran;
                    dir.push_back(i);
                }
                if (R.step == S_FIELD_DONE) fin.push_back(i);
            }
            if (!any_from && dir.empty() && fin.empty()) continue;
            upload_ctl(c_);
            hipStream_t s = c_->stream;
            if (any_from) launch_copy_state(c_->Mm.map, c_->d_(c_->from()), c_->st, c_->gprev, s);
            if (any_prec) {
                HIPCHK(hipEventRecord(c_->ev[2], s));
                const bool scaled = (ln_.mode & 2) && r_[0].scaled;
                precondition(c_, o_.jmax, scaled ? c_->dscale : nullptr, o_.precision == MM_FP32_BULK,
                             o_.prec_form);
                HIPCHK(hipEventRecord(c_->ev[3], s));
            }
            if (!dir.empty()) {
                launch_dir(c_->Mm.map, c_->d_(c_->act()), c_->d_(c_->first()), c_->st[0].g, c_->gprev, c_->y, c_->d,
                           mslot(c_, MS_DOTS), mslot(c_, MS_DOUT), c_->d_(c_->info()), o_.beta, c_->gy, s);
                launch_finalize_inst(c_->Mm.map, mslot(c_, MS_DOUT), 2, 2u, dsc_at(c_, SC_DIR), s);
                pull_sc(c_, SC_DIR, 2);
                pull_flags(c_);
            }
            if (!fin.empty() && out_.m_avg) {
                launch_mavg(c_->Mm.map, c_->st[0].x, c_->L, mslot(c_, MS_MISC), s);
                launch_finalize_inst(c_->Mm.map, mslot(c_, MS_MISC), 4, 0u, dsc_at(c_, SC_MISC), s);
                pull_sc(c_, SC_MISC, 4);
            }
            sync(c_);
            if (any_prec) {
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, c_->ev[2], c_->ev[3]));
                for (int i : dir)
                    if (r_[i].prec_ran) c_->cnt[i].t_lin += ms * 1e-3;
            }
            for (int i : fin) finish_field(i);
            for (int i : dir) after_dir(i);
        }
        return worst_;
    }

    const Sc &final_scalars(int i) const { return r_[i].cur; }
    long last_nli(int i) const { return r_[i].nli; }

private:
    mm_ctx *c_;
    const mm_opts &o_;
    const std::vector<double> &h_;
    long nf_;
    CurveOut out_;
    std::vector<Run> r_;
    Learned ln_;
    int worst_ = MM_OK;

    void start_field(int i, long k) {
        Run &R = r_[i];
        if (k >= nf_) {
            R.step = S_IDLE;
            return;
        }
        R.field = k;
        for (int q = 0; q < 3; ++q) R.h[q] = h_[(size_t)3 * (i * nf_ + k) + q];
        R.step = S_EVAL0;
        R.first = true;
        R.restarting = false;
        R.a_prev = R.dp_prev = 0.0;
        R.theta = o_.theta_max;
        R.nli = R.restarts = R.fallbacks = 0;
        R.c0 = c_->cnt[i];
        R.t0 = now_s();
        R.status = MM_NOT_CONVERGED;
        R.scaled = false;
        if (out_.accepted) out_.accepted[(size_t)i * nf_ + k] = 0;
    }

    void finish(int i, int status) {
        r_[i].status = status;
        r_[i].step = S_FIELD_DONE;
    }

    void need_dir(int i, int mode, bool restart) {
        Run &R = r_[i];
        R.dirmode = mode | (o_.jmax > 0 ? 0 : 2);
        R.restarting = restart;
        R.step = S_NEED_DIR;
    }

    void after_eval(int i, const Sc &v) {
        Run &R = r_[i];
        // a NaN or infinite energy (a breakdown somewhere in the evaluation)
        // ends the field; the accepted state is left as it was
        if (!std::isfinite(v.E)) return finish(i, MM_NONFINITE);
        switch (R.step) {
            case S_EVAL0:
                R.cur = v;
                if (o_.stop_mode == MM_STOP_TORQUE && v.tmax < o_.tol_torque) {
                    finish(i, MM_OK);
                } else if (ln_.mode && (R.field > 0 || ln_.has_prev)) {
                    // proposal of the network for this field step: start
                    // N(m + dm) and Jacobi factors s
                    const double *hp = R.field > 0 ? &h_[(size_t)3 * (i * nf_ + R.field - 1)] : ln_.h_prev;
                    gnn_propose(c_, ln_.net, ln_.graph, hp, R.h);
                    R.scaled = (ln_.mode & 2) != 0;
                    if (ln_.mode & 1) R.step = S_LEARN_T;
                    else need_dir(i, 1, false);
                } else {
                    need_dir(i, 1, false);
                }
                break;
            case S_LEARN_T:
                // energy-raise fallback: keep m_k unless the proposal is lower
                if (v.E < R.cur.E) {
                    c_->from()[i] = 1;
                    R.cur = v;
                    if (out_.accepted) out_.accepted[(size_t)i * nf_ + R.field] = 1;
                }
                if (o_.stop_mode == MM_STOP_TORQUE && R.cur.tmax < o_.tol_torque) finish(i, MM_OK);
                else need_dir(i, 1, false);
                break;
            case S_TRIAL_T: after_T(i, v); break;
            case S_TRIAL_C: after_C(i, v); break;
            case S_HALVE:
                if (v.dF <= o_.c1 * R.a * R.dp0) accept(i, 1, R.a, v);
                else halve(i);
                break;
            default: break;
        }
    }

    // line search on phi(alpha) = F(N(x + alpha d)): capped rotation (the cap
    // theta_max, or with theta_adapt the cap that follows the accepted steps),
    // sufficient decrease on the exact energy difference, one cubic
    // interpolation, then halving
    void start_ls(int i, double a0, bool restart) {
        Run &R = r_[i];
        R.restart_ls = restart;
        if (!(R.dmax > 0.0)) {
            ls_fail(i);
            return;
        }
        R.a0 = a0;
        R.amax = R.theta / R.dmax;
        R.at = std::min(a0, R.amax);
        R.step = S_TRIAL_T;
    }

    void after_T(int i, const Sc &v) {
        Run &R = r_[i];
        const double at = R.at, dp0 = R.dp0;
        R.sT = v;
        R.dFt = v.dF;
        R.arm_t = v.dF <= o_.c1 * at * dp0;
        if (R.arm_t && std::fabs(v.dphi) <= o_.c2 * std::fabs(dp0)) return accept(i, 1, at, v);
        const bool over = !R.arm_t || v.dphi > 0.0;
        if (!over && at >= R.amax) return accept(i, 1, at, v);
        double ac;
        if (!cubic_step(at, v.dF, dp0, v.dphi, &ac)) ac = over ? 0.5 * at : std::min(2.0 * at, R.amax);
        if (over) {
            ac = std::max(ac, 0.1 * at);
            ac = std::min(ac, 0.9 * at);
        } else {
            const double hi = std::min(4.0 * at, R.amax);
            ac = std::min(ac, hi);
            ac = std::max(ac, 1.1 * at);
            if (ac > hi) return accept(i, 1, at, v);
        }
        R.ac = ac;
        R.step = S_TRIAL_C;
    }

    void after_C(int i, const Sc &v) {
        Run &R = r_[i];
        if (v.dF <= o_.c1 * R.ac * R.dp0) return accept(i, 2, R.ac, v);
        if (R.arm_t) return accept(i, 1, R.at, R.sT);
        R.a = std::min(R.at, R.ac);
        R.halvings = 0;
        halve(i);
    }

    void halve(int i) {
        Run &R = r_[i];
        if (R.halvings >= o_.ls_max_halvings) return ls_fail(i);
        R.halvings++;
        R.a *= 0.5;
        R.step = S_HALVE;
    }

    void ls_fail(int i) {
        Run &R = r_[i];
        if (!R.restart_ls) {
            // restart along the steepest-descent direction
            R.restarts++;
            need_dir(i, 3, true);
        } else {
            finish(i, MM_STALLED);
        }
    }

    void accept(int i, int from, double alpha, const Sc &v) {
        Run &R = r_[i];
        c_->from()[i] = from;
        R.nli++;
        const Sc &s0 = R.cur;
        bool conv;
        if (o_.stop_mode == MM_STOP_TORQUE) {
            conv = v.tmax < o_.tol_torque;
        } else {
            const double tau = o_.tau_F;
            const bool t1 = (s0.E - v.E) < tau * (1.0 + std::fabs(v.E));
            const bool t2 = v.dxinf < std::sqrt(tau) * (1.0 + v.minf);
            const bool t3 = v.ginf < std::cbrt(tau) * (1.0 + std::fabs(v.E));
            conv = t1 && t2 && t3;
        }
        if (trace_level() > 0 && (R.nli <= 40 || R.nli % 100 == 0))
            std::fprintf(stderr,
                         "[mmncg] inst %d field %ld nli %ld alpha %.4e amax %.4e a0 %.4e dp0 %.4e dF %.4e dE %.4e "
                         "tmax %.4e E %.12e\n",
                         i, R.field, R.nli, alpha, R.amax, R.a0, R.dp0, v.dF, v.E - s0.E, v.tmax, v.E);
        R.cur = v;
        if (o_.theta_adapt) {
            // a step the cap stopped doubles it, a step below a quarter of it
            // halves it, within [theta_max, theta_hi]
            if (alpha >= R.amax * (1.0 - 1e-12)) R.theta = std::min(2.0 * R.theta, o_.theta_hi);
            else if (alpha < 0.25 * R.amax) R.theta = std::max(0.5 * R.theta, o_.theta_max);
        }
        if (conv) return finish(i, MM_OK);
        R.a_prev = alpha;
        R.dp_prev = R.dp0;
        R.first = false;
        need_dir(i, 0, false);
    }

    void after_dir(int i) {
        Run &R = r_[i];
        const double *r = hsc_at(c_, SC_DIR) + 2 * (size_t)i;
        R.dp0 = r[0];
        R.dmax = r[1];
        if (R.prec_ran) c_->cnt[i].li += c_->pflags()[4 * i + 1];
        if (R.restarting) {
            R.restarting = false;
            if (!(R.dp0 < 0.0) || !(R.dmax > 0.0)) return finish(i, MM_STALLED);
            return start_ls(i, o_.theta_init / R.dmax, true);
        }
        if (c_->info()[i] != 0) R.fallbacks++;
        // top of the nonlinear iteration
        if (R.nli >= o_.max_nli) return finish(i, MM_NOT_CONVERGED);
        // after the descent safeguard d = -g, so dp0 = -|g|^2: zero means a
        // zero projected gradient; a value that is not negative is NaN
        if (!(R.dp0 < 0.0)) return finish(i, R.dp0 == 0.0 ? MM_OK : MM_NONFINITE);
        double a0;
        if (R.first) a0 = o_.jmax > 0 ? 1.0 : o_.theta_init / R.dmax;
        else a0 = R.a_prev * R.dp_prev / R.dp0;
        start_ls(i, a0, false);
    }

    void finish_field(int i) {
        Run &R = r_[i];
        const long k = R.field;
        const size_t at = (size_t)i * nf_ + k;
        const Cnt &cn = c_->cnt[i];
        if (out_.st) {
            mm_stats &s = out_.st[at];
            s.evals = cn.evals - R.c0.evals;
            s.nli = R.nli;
            s.li = cn.li - R.c0.li;
            s.mi = cn.mi - R.c0.mi;
            s.restarts = R.restarts;
            s.fallbacks = R.fallbacks;
            s.t_nl = now_s() - R.t0;
            s.t_lin = cn.t_lin - R.c0.t_lin;
            s.t_mag = cn.t_mag - R.c0.t_mag;
            s.F = R.cur.E;
            s.torque_max = R.cur.tmax;
            s.status = R.status;
        }
        if (out_.m_avg) {
            const double *mv = hsc_at(c_, SC_MISC) + 4 * (size_t)i;
            for (int q = 0; q < 3; ++q) out_.m_avg[3 * at + q] = mv[q] / mv[3];
        }
        if (out_.E_tot) out_.E_tot[at] = R.cur.E;
        if (out_.m_hist && c_->ninst == 1) {
            const InstInfo &I = c_->inst[0];
            copy_out(c_, out_.m_hist + 3 * (size_t)I.n_mag * k, c_->st[0].x, 3 * (size_t)I.n_mag);
        }
        worst_ = std::max(worst_, R.status);
        start_field(i, k + 1);
    }
};

int precondition_call(mm_ctx *c, const double *m, const double *grad, const double *gproj, int jmax,
                      const double *dscale, double *y, int *inner_iters, const PrecScratch *ext) {
    require_single(c);
    if (!m || !grad || !gproj || !y || jmax < 0) throw ApiError{MM_EINVAL, "bad precondition arguments"};
    const int nm = c->inst[0].n_mag;
    load_m(c, m);
    copy_in(c, c->st[0].G, grad, 3 * (size_t)nm);
    copy_in(c, c->st[0].g, gproj, 3 * (size_t)nm);
    launch_lambda(c->Mm.map, c->st[0].x, c->st[0].G, c->st[0].lam, c->stream);
    int it = 0;
    if (jmax == 0) {
        HIPCHK(hipMemcpyAsync(c->y, c->st[0].g, 3 * (size_t)nm * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    } else {
        const double *ds = nullptr;
        if (dscale) {
            copy_in(c, c->dscale, dscale, nm);
            ds = c->dscale;
        }
        c->pact()[0] = 1;
        upload_ctl(c);
        precondition(c, jmax, ds, c->opts.precision == MM_FP32_BULK, c->opts.prec_form, ext);
        pull_prec_flags(c, ext ? ext->flags : c->d_(c->pflags()));
    }
    copy_out(c, y, c->y, 3 * (size_t)nm);
    sync(c);
    if (jmax > 0) it = c->pflags()[1];
    if (inner_iters) *inner_iters = it;
    return MM_OK;
}

bool opts_valid(const mm_opts &o, std::string &why) {
    if (o.jmax < 0) why = "jmax < 0";
    else if (!(o.tol_torque > 0)) why = "tol_torque <= 0";
    else if (!(o.theta_max > 0) || !(o.theta_init > 0)) why = "theta_max/theta_init <= 0";
    else if (o.theta_adapt != 0 && o.theta_adapt != 1) why = "theta_adapt not 0 or 1";
    else if (o.theta_adapt && !(o.theta_hi >= o.theta_max)) why = "theta_hi < theta_max";
    else if (!(o.c1 > 0 && o.c1 < 1) || !(o.c2 > o.c1 && o.c2 < 1)) why = "need 0 < c1 < c2 < 1";
    else if (!(o.poisson_rtol > 0)) why = "poisson_rtol <= 0";
    else if (o.max_nli < 1) why = "max_nli < 1";
    else if (o.precision != MM_FP64 && o.precision != MM_FP32_BULK) why = "unknown precision";
    else if (o.stop_mode != MM_STOP_TORQUE && o.stop_mode != MM_STOP_PAPER) why = "unknown stop_mode";
    else if (o.stop_mode == MM_STOP_PAPER && !(o.tau_F > 0)) why = "tau_F <= 0";
    else if (o.poisson_maxit < 1) why = "poisson_maxit < 1";
    else if (o.ls_max_halvings < 0) why = "ls_max_halvings < 0";
    else if (o.poisson_prec != MM_PREC_JACOBI && o.poisson_prec != MM_PREC_AMG) why = "unknown poisson_prec";
    else if (o.beta < MM_BETA_ZA || o.beta > MM_BETA_HS) why = "unknown beta";
    else if (o.prec_form < MM_PFORM_PAPER || o.prec_form > MM_PFORM_LOCAL) why = "unknown prec_form";
    else return true;
    return false;
}

mm_opts resolve_opts(const mm_opts *o) {
    mm_opts op;
    if (o) op = *o;
    else mm_opts_default(&op);
    std::string why;
    if (!opts_valid(op, why)) throw ApiError{MM_EINVAL, why};
    return op;
}

void require_ready(mm_ctx *c) {
    if (!c->have_mat || c->ninst < 1) throw ApiError{MM_ESTATE, "mesh and material must be set first"};
}
void require_single(mm_ctx *c) {
    require_ready(c);
    if (c->ninst != 1) throw ApiError{MM_ESTATE, "this call needs a context with exactly one instance"};
}

// evaluation of every instance at the current state for fields h (reduced, [inst][3])
void eval_all(mm_ctx *c, const mm_opts &o, const std::vector<double> &h) {
    std::vector<int> on;
    for (int i = 0; i < c->ninst; ++i) {
        c->act()[i] = 1;
        c->role()[i] = 0;
        c->alpha()[i] = 0.0;
        set_h3(c, i, &h[3 * (size_t)i]);
        on.push_back(i);
    }
    eval_round(c, o, on, false);
}

// check mesh arrays of one instance
void check_mesh(const double *xyz, long n_nodes, const int *tets, long n_tets) {
    if (!xyz || !tets || n_nodes < 4 || n_tets < 1) throw ApiError{MM_EINVAL, "bad mesh arguments"};
    for (long e = 0; e < 4 * n_tets; ++e)
        if (tets[e] < 0 || tets[e] >= n_nodes) throw ApiError{MM_EMESH, "tet node index out of range"};
    for (long i = 0; i < 3 * n_nodes; ++i)
        if (!std::isfinite(xyz[i])) throw ApiError{MM_EMESH, "non-finite coordinate"};
}

Assembly assemble_checked(const double *xyz, long n_nodes, const int *tets, long n_tets, const int *region,
                          const double *Ms, const double *A, const double *K1, const double *axis, int inst) {
    Assembly as;
    std::string e = assemble(xyz, n_nodes, tets, n_tets, region, Ms, A, K1, axis, as);
    std::string where = inst >= 0 ? " (instance " + std::to_string(inst) + ")" : "";
    if (!e.empty()) throw ApiError{MM_EMESH, e + where};
    if (as.n_mag == 0) throw ApiError{MM_EMESH, "no magnet nodes" + where};
    for (int a = 0; a < as.n_mag; ++a)
        if (!(as.Dex[a] > 0.0)) throw ApiError{MM_EMESH, "zero exchange diagonal at a magnet node" + where};
    return as;
}

}  // namespace mmncg

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int mm_opts_default(mm_opts *o) {
    if (!o) return MM_EINVAL;
    std::memset(o, 0, sizeof *o);
    o->jmax = 4;
    o->tol_torque = 1e-6;
    o->stop_mode = MM_STOP_TORQUE;
    o->tau_F = 1e-10;
    o->theta_max = 0.2;
    o->theta_init = 0.01;
    o->c1 = 1e-4;
    o->c2 = 0.1;
    o->poisson_rtol = 1e-10;
    o->max_nli = 20000;
    o->precision = MM_FP64;
    o->terms = MM_T_ALL;
    o->ls_max_halvings = 20;
    o->poisson_maxit = 100000;
    o->poisson_prec = MM_PREC_JACOBI;
    o->beta = MM_BETA_ZA;
    o->prec_form = MM_PFORM_PAPER;
    o->theta_adapt = 0;
    o->theta_hi = 1.5707963267948966;
    return MM_OK;
}

int mm_create(mm_ctx **out, int device, void *hip_stream, mm_alloc_fn dev_alloc, mm_free_fn dev_free,
              void *alloc_user) {
    if (!out) return MM_EINVAL;
    *out = nullptr;
    if ((dev_alloc == nullptr) != (dev_free == nullptr)) return MM_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return MM_EDEVICE;
    }
    mm_ctx *c = new (std::nothrow) mm_ctx();
    if (!c) return MM_ENOMEM;
    c->device = device;
    c->ualloc = dev_alloc;
    c->ufree = dev_free;
    c->user = alloc_user;
    mm_opts_default(&c->opts);
    int rc = guarded(c, [&] {
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        for (auto &e : c->ev) HIPCHK(hipEventCreate(&e));
        return MM_OK;
    });
    if (rc != MM_OK) {
        mm_destroy(c);
        return rc;
    }
    *out = c;
    return MM_OK;
}

int mm_destroy(mm_ctx *c) {
    if (!c) return MM_EINVAL;
    (void)hipSetDevice(c->device);
    free_all(c);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->prof_ev) (void)hipEventDestroy(e);
    for (auto &v : c->kt_ev)
        for (auto &e : v) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return MM_OK;
}

const char *mm_last_error(const mm_ctx *c) { return c ? c->err.c_str() : "null context"; }

int mm_get_info(const mm_ctx *c, mm_info *info) {
    if (!c || !info) return MM_EINVAL;
    std::memset(info, 0, sizeof *info);
    if (!c->have_mat) {
        info->n_nodes = (long)c->xyz.size() / 3;
        info->n_tets = (long)c->tets.size() / 4;
        return MM_OK;
    }
    for (const InstInfo &I : c->inst) {
        info->n_nodes += I.n_nodes;
        info->n_tets += I.n_tets;
        info->n_mag += I.n_mag;
        info->n_pot += I.n_pot;
        info->nnz_C_blocks += I.nnz_C;
        info->nnz_K += I.nnz_K;
        info->nnz_B += I.nnz_B;
    }
    info->Ms_ref = c->inst.empty() ? 0.0 : c->inst[0].Ms_ref;
    info->device_bytes = c->dev_bytes;
    return MM_OK;
}

int mm_mesh_upload(mm_ctx *c, const double *xyz, long n_nodes, const int *tets, long n_tets, const int *region) {
    return guarded(c, [&] {
        if (!region) throw ApiError{MM_EINVAL, "bad mesh arguments"};
        check_mesh(xyz, n_nodes, tets, n_tets);
        if (is_device_ptr(xyz) || is_device_ptr(tets) || is_device_ptr(region))
            throw ApiError{MM_EINVAL, "mesh arrays must be host memory"};
        free_all(c);
        c->xyz.assign(xyz, xyz + 3 * n_nodes);
        c->tets.assign(tets, tets + 4 * n_tets);
        c->region.assign(region, region + n_tets);
        c->have_mesh = true;
        c->have_mat = false;
        return MM_OK;
    });
}

int mm_material_set(mm_ctx *c, const double *Ms, const double *A, const double *K1, const double *axis) {
    return guarded(c, [&] {
        if (!c->have_mesh) throw ApiError{MM_ESTATE, "upload the mesh first"};
        if (!Ms || !A || !K1) throw ApiError{MM_EINVAL, "Ms, A and K1 are required"};
        const long nn = (long)c->xyz.size() / 3, nt = (long)c->tets.size() / 4;
        std::vector<Assembly> as;
        as.push_back(assemble_checked(c->xyz.data(), nn, c->tets.data(), nt, c->region.data(), Ms, A, K1, axis, -1));
        c->have_mat = false;
        setup_device(c, as, {nn}, {nt});
        c->have_mat = true;
        return MM_OK;
    });
}

int mm_batch_upload(mm_ctx *c, int n_inst, const long *n_nodes, const long *n_tets, const double *xyz,
                    const int *tets, const int *region, const double *Ms, const double *A, const double *K1,
                    const double *axis) {
    return guarded(c, [&] {
        if (n_inst < 1 || !n_nodes || !n_tets || !xyz || !tets || !region || !Ms || !A || !K1)
            throw ApiError{MM_EINVAL, "bad batch arguments"};
        for (const void *p : {(const void *)xyz, (const void *)tets, (const void *)region, (const void *)Ms,
                              (const void *)A, (const void *)K1, (const void *)axis})
            if (is_device_ptr(p)) throw ApiError{MM_EINVAL, "batch arrays must be host memory"};
        std::vector<Assembly> as;
        std::vector<long> nn(n_inst), nt(n_inst);
        long on = 0, ot = 0;
        for (int i = 0; i < n_inst; ++i) {
            nn[i] = n_nodes[i];
            nt[i] = n_tets[i];
            if (nn[i] < 4 || nt[i] < 1) throw ApiError{MM_EINVAL, "bad mesh size of instance " + std::to_string(i)};
            check_mesh(xyz + 3 * on, nn[i], tets + 4 * ot, nt[i]);
            as.push_back(assemble_checked(xyz + 3 * on, nn[i], tets + 4 * ot, nt[i], region + ot, Ms + ot, A + ot,
                                          K1 + ot, axis ? axis + 3 * ot : nullptr, i));
            on += nn[i];
            ot += nt[i];
        }
        free_all(c);
        c->xyz.clear();
        c->tets.clear();
        c->region.clear();
        c->have_mesh = true;
        c->have_mat = false;
        setup_device(c, as, nn, nt);
        c->have_mat = true;
        return MM_OK;
    });
}

int mm_batch_info(const mm_ctx *c, int inst, mm_info *info) {
    if (!c || !info) return MM_EINVAL;
    if (!c->have_mat) return MM_ESTATE;
    if (inst < 0 || inst >= c->ninst) return MM_EINVAL;
    const InstInfo &I = c->inst[inst];
    std::memset(info, 0, sizeof *info);
    info->n_nodes = I.n_nodes;
    info->n_tets = I.n_tets;
    info->n_mag = I.n_mag;
    info->n_pot = I.n_pot;
    info->nnz_C_blocks = I.nnz_C;
    info->nnz_K = I.nnz_K;
    info->nnz_B = I.nnz_B;
    info->Ms_ref = I.Ms_ref;
    info->device_bytes = c->dev_bytes;
    return MM_OK;
}

int mm_batch_size(const mm_ctx *c, int *n_inst) {
    if (!c || !n_inst) return MM_EINVAL;
    *n_inst = c->have_mat ? c->ninst : 0;
    return MM_OK;
}

int mm_batch_magnet_nodes(const mm_ctx *c, int inst, long *n_mag, int *node_ids) {
    if (!c || !n_mag) return MM_EINVAL;
    if (!c->have_mat) return MM_ESTATE;
    if (inst < 0 || inst >= c->ninst) return MM_EINVAL;
    const InstInfo &I = c->inst[inst];
    *n_mag = I.n_mag;
    if (node_ids) std::memcpy(node_ids, I.node_of_mag.data(), sizeof(int) * I.n_mag);
    return MM_OK;
}

int mm_magnet_nodes(const mm_ctx *c, long *n_mag, int *node_ids) {
    if (!c || !n_mag) return MM_EINVAL;
    if (!c->have_mat) return MM_ESTATE;
    if (c->ninst != 1) return MM_ESTATE;
    return mm_batch_magnet_nodes(c, 0, n_mag, node_ids);
}

int mm_set_opts(mm_ctx *c, const mm_opts *o) {
    return guarded(c, [&] {
        if (!o) throw ApiError{MM_EINVAL, "null opts"};
        c->opts = resolve_opts(o);
        return MM_OK;
    });
}

int mm_reset_warm_start(mm_ctx *c) {
    return guarded(c, [&] {
        require_ready(c);
        launch_fill(c->rows_p, c->u, 0.0, c->stream);
        sync(c);
        c->last_pcg.assign((size_t)kPcgKinds * c->ninst, 16);
        return MM_OK;
    });
}

int mm_energy_grad(mm_ctx *c, const double *m, const double h_ext[3], double E_parts[5], double *grad, double *gproj,
                   double *torque_max) {
    return guarded(c, [&] {
        require_single(c);
        if (!m || !h_ext) throw ApiError{MM_EINVAL, "m and h_ext are required"};
        load_m(c, m);
        std::vector<double> h(3);
        reduce_field(c->inst[0], h_ext, h.data());
        eval_all(c, c->opts, h);
        const Sc v = eval_result(c, 0);
        const size_t n3 = 3 * (size_t)c->inst[0].n_mag;
        if (E_parts) energy_parts(c, 0, v, c->opts, E_parts);
        if (grad) copy_out(c, grad, c->st[0].G, n3);
        if (gproj) copy_out(c, gproj, c->st[0].g, n3);
        if (torque_max) *torque_max = v.tmax;
        sync(c);
        return MM_OK;
    });
}

int mm_batch_energy_grad(mm_ctx *c, const double *m, const double *h_ext, double *E_tot, double *grad, double *gproj,
                         double *torque_max) {
    return guarded(c, [&] {
        require_ready(c);
        if (!m || !h_ext) throw ApiError{MM_EINVAL, "m and h_ext are required"};
        load_m(c, m);
        std::vector<double> h(3 * (size_t)c->ninst);
        for (int i = 0; i < c->ninst; ++i) reduce_field(c->inst[i], h_ext + 3 * i, &h[3 * (size_t)i]);
        eval_all(c, c->opts, h);
        for (int i = 0; i < c->ninst; ++i) {
            const Sc v = eval_result(c, i);
            if (E_tot) E_tot[i] = v.E;
            if (torque_max) torque_max[i] = v.tmax;
        }
        for (const InstInfo &I : c->inst) {
            if (grad) copy_out(c, grad + 3 * I.user_off, c->st[0].G + 3 * (size_t)I.mag_off, 3 * (size_t)I.n_mag);
            if (gproj) copy_out(c, gproj + 3 * I.user_off, c->st[0].g + 3 * (size_t)I.mag_off, 3 * (size_t)I.n_mag);
        }
        sync(c);
        return MM_OK;
    });
}

int mm_precondition(mm_ctx *c, const double *m, const double *grad, const double *gproj, int jmax, const double *dscale,
                    double *y, int *inner_iters) {
    return guarded(c, [&] { return precondition_call(c, m, grad, gproj, jmax, dscale, y, inner_iters, nullptr); });
}

int mm_ncg_minimize(mm_ctx *c, double *m_inout, const double h_ext[3], const mm_opts *o, mm_stats *st,
                    double E_parts[5]) {
    return guarded(c, [&] {
        require_single(c);
        if (!m_inout || !h_ext) throw ApiError{MM_EINVAL, "m and h_ext are required"};
        mm_opts op = resolve_opts(o);
        load_m(c, m_inout);
        std::vector<double> h(3);
        reduce_field(c->inst[0], h_ext, h.data());
        mm_stats s;
        CurveOut out;
        out.st = &s;
        Driver drv(c, op, h, 1, out);
        int rc = drv.run();
        if (E_parts) energy_parts(c, 0, drv.final_scalars(0), op, E_parts);
        store_m(c, m_inout);
        sync(c);
        if (st) *st = s;
        return rc;
    });
}

int mm_demag_curve(mm_ctx *c, double *m_inout, const double *h_list, long n, const mm_opts *o, double *m_avg,
                   double *E_tot, mm_stats *st, double *m_hist) {
    return guarded(c, [&] {
        require_single(c);
        if (!m_inout || !h_list || n < 0) throw ApiError{MM_EINVAL, "bad curve arguments"};
        mm_opts op = resolve_opts(o);
        load_m(c, m_inout);
        std::vector<double> h(3 * (size_t)n);
        for (long k = 0; k < n; ++k) reduce_field(c->inst[0], h_list + 3 * k, &h[3 * k]);
        CurveOut out;
        out.m_avg = m_avg;
        out.E_tot = E_tot;
        out.st = st;
        out.m_hist = m_hist;
        Driver drv(c, op, h, n, out);
        int rc = drv.run();
        store_m(c, m_inout);
        sync(c);
        return rc;
    });
}

int mm_batch_demag_curve(mm_ctx *c, double *m_inout, const double *h_list, long n, const mm_opts *o, double *m_avg,
                         double *E_tot, mm_stats *st) {
    return guarded(c, [&] {
        require_ready(c);
        if (!m_inout || !h_list || n < 0) throw ApiError{MM_EINVAL, "bad curve arguments"};
        mm_opts op = resolve_opts(o);
        load_m(c, m_inout);
        const int ni = c->ninst;
        std::vector<double> h(3 * (size_t)n * ni);
        for (int i = 0; i < ni; ++i)
            for (long k = 0; k < n; ++k) {
                const size_t at = 3 * ((size_t)i * n + k);
                reduce_field(c->inst[i], h_list + at, &h[at]);
            }
        CurveOut out;
        out.m_avg = m_avg;
        out.E_tot = E_tot;
        out.st = st;
        Driver drv(c, op, h, n, out);
        int rc = drv.run();
        store_m(c, m_inout);
        sync(c);
        return rc;
    });
}

int mm_demag_curve_learned(mm_ctx *c, mm_gnn *net, mm_graph *graph, int mode, double *m_inout,
                           const double *h_prev, const double *h_list, long n, const mm_opts *o, double *m_avg,
                           double *E_tot, mm_stats *st, int *accepted) {
    return guarded(c, [&] {
        require_single(c);
        if (!m_inout || !h_list || n < 0) throw ApiError{MM_EINVAL, "bad curve arguments"};
        if (mode < 0 || mode > 3) throw ApiError{MM_EINVAL, "unknown learned mode"};
        if (mode && (!net || !graph)) throw ApiError{MM_EINVAL, "network and graph are required"};
        mm_opts op = resolve_opts(o);
        load_m(c, m_inout);
        std::vector<double> h(3 * (size_t)n);
        for (long k = 0; k < n; ++k) reduce_field(c->inst[0], h_list + 3 * k, &h[3 * k]);
        CurveOut out;
        out.m_avg = m_avg;
        out.E_tot = E_tot;
        out.st = st;
        out.accepted = accepted;
        Learned ln;
        ln.net = net;
        ln.graph = graph;
        ln.mode = mode;
        if (h_prev) {
            ln.has_prev = true;
            reduce_field(c->inst[0], h_prev, ln.h_prev);
        }
        Driver drv(c, op, h, n, out, ln);
        int rc = drv.run();
        store_m(c, m_inout);
        sync(c);
        return rc;
    });
}

int mm_operator_apply(mm_ctx *c, int op, const double *in, double *out) {
    return guarded(c, [&] {
        require_single(c);
        if (!in || !out) throw ApiError{MM_EINVAL, "null vector"};
        const int nm = c->inst[0].n_mag, np = c->inst[0].n_pot;
        const bool fp32 = c->opts.precision == MM_FP32_BULK;
        hipStream_t s = c->stream;
        switch (op) {
            case MM_OP_C:
                copy_in(c, c->tmp3, in, 3 * (size_t)nm);
                launch_spmv_block6(c->C, c->Mm.map, c->tmp3, c->pq, fp32, s);
                copy_out(c, out, c->pq, 3 * (size_t)nm);
                break;
            case MM_OP_B: {
                copy_in(c, c->tmp3, in, 3 * (size_t)nm);
                launch_fill(np, c->cq, 0.0, s);
                StateV sv[3];
                sv[0].x = c->tmp3;
                launch_bmul(c->B, c->Mb.map, nullptr, sv, nullptr, c->cq, fp32, s);
                pot_out(c, out, c->cq, c->cr);
                break;
            }
            case MM_OP_BT:
                pot_in(c, c->cq, in, c->cr);
                launch_btmul(c->Bt, c->Mm.map, c->cq, c->pq, fp32, s);
                copy_out(c, out, c->pq, 3 * (size_t)nm);
                break;
            case MM_OP_K:
                pot_in(c, c->cr, in, c->cq);
                launch_spmv_scalar(c->K, c->Mp.map, c->cr, c->cq, fp32, s);
                pot_out(c, out, c->cq, c->cr);
                break;
            default:
                throw ApiError{MM_EINVAL, "unknown operator"};
        }
        sync(c);
        return MM_OK;
    });
}

int mm_poisson_solve(mm_ctx *c, const double *b, double *u_inout, double rtol, long *iters) {
    return guarded(c, [&] {
        require_single(c);
        if (!b || !u_inout || !(rtol > 0)) throw ApiError{MM_EINVAL, "bad Poisson arguments"};
        const int np = c->inst[0].n_pot;
        // the solve runs on the context's b and u: keep the warm start aside
        HIPCHK(hipMemcpyAsync(c->usave, c->u, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        // evaluations write only the magnet rows of b, so b is cleared and the
        // warm start restored on every exit, failed solves included
        auto restore = [&] {
            launch_fill(np, c->b, 0.0, c->stream);
            HIPCHK(hipMemcpyAsync(c->u, c->usave, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            sync(c);
        };
        long it = 0;
        try {
            pot_in(c, c->b, b, c->cq);
            pot_in(c, c->u, u_inout, c->cq);
            c->act()[0] = 1;
            upload_ctl(c);
            const long mi0 = c->cnt[0].mi;
            poisson(c, rtol, c->opts.poisson_maxit, c->opts.precision == MM_FP32_BULK,
                    c->opts.poisson_prec == MM_PREC_AMG, {0});
            it = c->cnt[0].mi - mi0;
            pot_out(c, u_inout, c->u, c->cq);
        } catch (const ApiError &e) {
            // not converged within poisson_maxit: the last iterate is the result
            if (e.code == MM_NOT_CONVERGED) pot_out(c, u_inout, c->u, c->cq);
            restore();
            throw;
        } catch (...) {
            restore();
            throw;
        }
        restore();
        if (iters) *iters = it;
        return MM_OK;
    });
}

int mm_tune(mm_ctx *c, int mode, const char *cache_path, int *waves_per_block, int *slices_per_wave,
            int *block_mult) {
    return guarded(c, [&] {
        require_ready(c);
        const bool fp32 = c->opts.precision == MM_FP32_BULK;
        switch (mode) {
            case MM_TUNE_DEFAULT:
                set_poisson_shape(c, kPoissonWaves, std::vector<int>(c->ninst, 1));
                c->tuned = false;
                break;
            case MM_TUNE_MEASURE:
                autotune(c, false, nullptr, fp32);
                break;
            case MM_TUNE_CACHE:
                if (!cache_path) throw ApiError{MM_EINVAL, "cache_path is required"};
                autotune(c, true, cache_path, fp32);
                break;
            default:
                throw ApiError{MM_EINVAL, "unknown tuning mode"};
        }
        if (waves_per_block) *waves_per_block = c->pnw;
        if (block_mult) *block_mult = c->pbm;
        if (slices_per_wave)
            for (int i = 0; i < c->ninst; ++i) slices_per_wave[i] = c->pspw[i];
        return MM_OK;
    });
}

int mm_profile_kernels(mm_ctx *c, int enable, double out[9]) {
    return guarded(c, [&] {
        if (c->stream) sync(c);
        kt_harvest(c);
        if (enable < 0) {
            for (int k = 0; k < KT_N; ++k) c->kt_sec[k] = c->kt_calls[k] = c->kt_bytes[k] = 0;
        } else {
            c->kt_on = enable != 0;
        }
        if (out)
            for (int k = 0; k < KT_N; ++k) {
                out[3 * k] = c->kt_calls[k];
                out[3 * k + 1] = c->kt_sec[k];
                out[3 * k + 2] = c->kt_bytes[k];
            }
        return MM_OK;
    });
}

int mm_profile(mm_ctx *c, int enable, double out[4]) {
    return guarded(c, [&] {
        if (c->stream) sync(c);
        prof_harvest(c);
        if (enable < 0) {
            c->prof_seconds = c->prof_units = c->prof_bytes = 0;
        } else {
            c->prof_on = enable != 0;
        }
        if (out) {
            out[0] = c->prof_units;
            out[1] = c->prof_seconds;
            out[2] = c->prof_bytes;
            double rows = 0;
            for (const InstInfo &I : c->inst) rows += I.n_pot;
            out[3] = rows;
        }
        return MM_OK;
    });
}

}  // extern "C"
