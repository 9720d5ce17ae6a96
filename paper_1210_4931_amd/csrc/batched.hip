// Batched FP32 path: many right-hand sides share one plan and the Legendre steps become
// dense contractions on the matrix cores (MFMA), the GPU form of the transforms that
// Sect. 3 names as the cost driver.
//
// For one m, with columns c = (map, re/im) of all maps in the batch:
//   synthesis  E[p][c] = sum_{l+m even} lambda_lm(z_p) s'[l][c],  O likewise over odd l+m,
//              F_N = E + O, F_S = E - O                      ([pairs x L] x [L x cols])
//   analysis   a[l][c] = sum_p lambda_lm(z_p) X_{(l+m) mod 2}[p][c],
//              X_0 = G_N + G_S, X_1 = G_N - G_S              ([L x pairs] x [pairs x cols])
// lambda_lm is tabulated once per plan in FP32 (computed from the FP64 recurrence and start
// seeds, zero below each pair's start index), as rows [m][pair][l - m] padded to 128 values of
// l and 64 pairs.  The products run on v_mfma_f32_32x32x2f32 with FP32 accumulation; the
// ring-Fourier array ([ring][m][cols]) and the coefficients ([alm][cols]) are FP32 with the
// maps innermost, so tiles of columns are contiguous.  Maps, the pixel update and every
// diagnostic stay FP64.  The ring FFTs are the FP64 transforms of the per-map path with
// FP32 per-map output rows, regrouped into the column layout by LDS-tiled transposes.
#include "fft_core.h"

namespace mfwf {

typedef float floatx16 __attribute__((ext_vector_type(16)));
// Native 4-vectors for the prefetch registers: copies of the HIP float4 struct into LDS are
// aggregate copies that keep the source array in scratch memory.
typedef float floatx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------------------
// lambda table: one lane per ring pair, one workgroup per (pair tile of 64, m).
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(64)
k_lam_table(const double *__restrict__ Atab, const double *__restrict__ ctab,
            const long *__restrict__ mofs, const int *__restrict__ lstart,
            const double2 *__restrict__ seed, const double *__restrict__ zp,
            const long *__restrict__ loff, const int *__restrict__ Lp, float *__restrict__ lam,
            int lmax, int npair) {
    const int p = blockIdx.x * 64 + threadIdx.x, m = blockIdx.y;
    const int L = Lp[m];
    float *row = lam + loff[m] + (long)p * L;
    const long off = mofs[m] - m;
    if (p >= npair) {
        for (int r = 0; r < L; r++) row[r] = 0.f;
        return;
    }
    const int ls = lstart[(long)m * npair + p];
    const double2 sd = seed[(long)m * npair + p];
    const double z = zp[p];
    double u1 = 0.0, u2 = 0.0;
    for (int r = 0; r < L; r++) {
        const int l = m + r;
        float v = 0.f;
        if (l <= lmax && l >= ls) {
            double mu;
            if (l == ls) {
                mu = sd.y;
                u1 = sd.x;
            } else {
                mu = fma(Atab[off + l] * z, u1, -u2);
            }
            u2 = u1;
            u1 = mu;
            v = (float)(ctab[off + l] * mu);  // lambda = c mu
        }
        row[r] = v;
    }
}

// ---------------------------------------------------------------------------------------
// lambda rows generated inside the GEMMs (temperature batched form): instead of reading
// the FP32 table the GEMMs run the FP64 recurrence of k_lam_table themselves, 16 rows at a
// time, from its state at the start of every 16-row segment of a row, tabulated once per
// plan (16 bytes per 16 table entries: a quarter of the table's size, and the only
// per-(m, pair, l) data the GEMMs read).  The arithmetic and its order are k_lam_table's,
// so the generated values equal the table's bit for bit.
// ---------------------------------------------------------------------------------------
// lck[(segoff[m] + s) Rp + p] = (mu_{l-1}, mu_{l-2}) entering row l = m + 16 s of pair p,
// zero before the pair's start index (and for the padding pairs)
__global__ void __launch_bounds__(64)
k_lam_ckpt(const double *__restrict__ Atab, const long *__restrict__ mofs,
           const int *__restrict__ lstart, const double2 *__restrict__ seed,
           const double *__restrict__ zp, const int *__restrict__ Lp,
           const long *__restrict__ segoff, double2 *__restrict__ lck, int lmax, int npair,
           int Rp) {
    const int p = blockIdx.x * 64 + threadIdx.x, m = blockIdx.y;
    const int L = Lp[m];
    double2 *out = lck + segoff[m] * Rp + p;
    if (p >= npair) {
        for (int r = 0; r < L; r += 16) out[(long)(r / 16) * Rp] = make_double2(0.0, 0.0);
        return;
    }
    const long off = mofs[m] - m;
    const int ls = lstart[(long)m * npair + p];
    const double2 sd = seed[(long)m * npair + p];
    const double z = zp[p];
    double u1 = 0.0, u2 = 0.0;
    for (int r = 0; r < L; r++) {
        if ((r & 15) == 0) out[(long)(r / 16) * Rp] = make_double2(u1, u2);
        const int l = m + r;
        if (l <= lmax && l >= ls) {
            double mu;
            if (l == ls) {
                mu = sd.y;
                u1 = sd.x;
            } else {
                mu = fma(Atab[off + l] * z, u1, -u2);
            }
            u2 = u1;
            u1 = mu;
        }
    }
}

// Rows l0 .. l0 + 15 of one pair from the segment state st = (u1, u2): the steps of
// k_lam_table; A(r), c(r) give the coefficients A_lm, c_lm of row l0 + r; sink(q, v4)
// receives rows 4 q .. 4 q + 3 as they are ready.
template <typename FA, typename FC, typename FS>
__device__ __forceinline__ void lam_rows16(double2 st, int ls, double2 sd, double z, int l0,
                                           int lmax, FA A, FC c, FS sink) {
    double u1 = st.x, u2 = st.y;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int r = 4 * q + i, l = l0 + r;
            float x = 0.f;
            if (l <= lmax && l >= ls) {
                double mu;
                if (l == ls) {
                    mu = sd.y;
                    u1 = sd.x;
                } else {
                    mu = fma(A(r) * z, u1, -u2);
                }
                u2 = u1;
                u1 = mu;
                x = (float)(c(r) * mu);
            }
            v[i] = x;
        }
        sink(q, v);
    }
}

// what a GEMM needs to generate its lambda rows
struct LamGen {
    const double2 *lck;    // segment states (k_lam_ckpt)
    const long *segoff;    // [nm] first segment of each m
    const int *lstart;     // [nm][npair]
    const double2 *seed;   // [nm][npair]
    const double *z;       // [npair]
    const double *A, *c;   // [nalm]
};

// ---------------------------------------------------------------------------------------
// Layout changes between the per-map ring-Fourier rows of the ring transforms,
// [map][ring][m] (FP32 complex), and the contraction layout [m][ring][C2] with columns 2b
// (re) and 2b + 1 (im) of map b.  One workgroup moves a tile of 64 values of m x 64 maps
// of one ring through LDS, so that both sides read and write 512-byte rows.  Each thread
// issues all of its 16 loads before it stores any of them (clamped in-range addresses, values
// selected), so that a workgroup has its whole tile in flight at once.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_rows_to_cols(const float2 *__restrict__ phf, float *__restrict__ ph32, int nring, int nm,
               int rs, int nb, int Bp, int C2) {
    __shared__ float2 tile[64][64 + 1];  // [map][m]
    const int ring = blockIdx.x, m0 = 64 * blockIdx.y, b0 = 64 * blockIdx.z;
    float2 v[16];
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const int e = threadIdx.x + 256 * u, bb = e >> 6, mm = e & 63, b = b0 + bb, m = m0 + mm;
        const float2 x = phf[((long)min(b, nb - 1) * nring + ring) * rs + min(m, nm - 1)];
        v[u] = (b < nb && m < nm) ? x : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const int e = threadIdx.x + 256 * u;
        tile[e >> 6][e & 63] = v[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const int e = threadIdx.x + 256 * u, mm = e >> 6, bb = e & 63, b = b0 + bb, m = m0 + mm;
        if (b < Bp && m < nm)
            *reinterpret_cast<float2 *>(ph32 + ((long)m * nring + ring) * C2 + 2 * b) = tile[bb][mm];
    }
}

// map b's two columns (2b, 2b + 1) of every (m, ring) row of the columns [m][ring][C2] set
// to zero: a map whose chained iterations start from s = 0
__global__ void __launch_bounds__(256)
k_zero_map_cols(float *__restrict__ ph32, long nrows, int C2, int b) {
    for (long i = blockIdx.x * 256L + threadIdx.x; i < nrows; i += (long)gridDim.x * 256)
        *reinterpret_cast<float2 *>(ph32 + i * C2 + 2 * b) = make_float2(0.f, 0.f);
}

__global__ void __launch_bounds__(256)
k_cols_to_rows(const float *__restrict__ ph32, float2 *__restrict__ phf, int nring, int nm,
               int rs, int nb, int C2) {
    __shared__ float2 tile[64][64 + 1];  // [m][map]
    const int ring = blockIdx.x, m0 = 64 * blockIdx.y, b0 = 64 * blockIdx.z;
    float2 v[16];
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const int e = threadIdx.x + 256 * u, mm = e >> 6, bb = e & 63, b = b0 + bb, m = m0 + mm;
        const float2 x = *reinterpret_cast<const float2 *>(
            ph32 + ((long)min(m, nm - 1) * nring + ring) * C2 + 2 * min(b, nb - 1));
        v[u] = (b < nb && m < nm) ? x : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const int e = threadIdx.x + 256 * u;
        tile[e >> 6][e & 63] = v[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const int e = threadIdx.x + 256 * u, bb = e >> 6, mm = e & 63, b = b0 + bb, m = m0 + mm;
        if (b < nb && m < nm) phf[((long)b * nring + ring) * rs + m] = tile[mm][bb];
    }
}

// ---------------------------------------------------------------------------------------
// MFMA GEMMs.  Workgroup of 4 waves.  v_mfma_f32_32x32x2f32 operands: A[i][k] in lane
// i + 32k, B[k][j] in lane j + 32k; accumulator register r of lane L holds
// D[8 (r/4) + 4 (L/32) + r%4][L%32].
//
// Workgroup i of a launch is dispatched to XCD i mod 8.  Each XCD takes its tiles from its
// own list, so that all tiles of one m, which read the same ring-Fourier (analysis) or
// coefficient (synthesis) block, run on one XCD and share its L2 instead of fetching the
// block from HBM once per XCD; the lists are balanced by the number of active K chunks.
// Global loads of the next K chunk are issued before the matrix products of the current
// one (register double buffering).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// Tile of workgroup bid: XCD x = bid mod 8 works through its own list tab[x][*] of tiles
// (balanced by work on the host, tiles of one m adjacent); columns groups innermost.
struct XcdTile {
    int item, cg;
};
__device__ __forceinline__ XcdTile xcd_tile(const int *__restrict__ tab, int per_xcd, int ncg) {
    const int x = blockIdx.x & 7, s = blockIdx.x >> 3;
    const int k = s / ncg;
    XcdTile r;
    r.cg = s - k * ncg;
    r.item = (k < per_xcd) ? tab[x * per_xcd + k] : -1;
    return r;
}

__device__ __forceinline__ floatx4 ld4(const float *q) { return *reinterpret_cast<const floatx4 *>(q); }
__device__ __forceinline__ void st4(float *q, floatx4 v) { *reinterpret_cast<floatx4 *>(q) = v; }
// v if c, else zeros (a value select; a conditional load would become a load through a
// selected pointer and force a stack copy)
__device__ __forceinline__ floatx4 keep4(bool c, floatx4 v) { return c ? v : floatx4{0.f, 0.f, 0.f, 0.f}; }

// threadIdx.x read anew: an epilogue that forms its lane indices from it keeps them out of
// the registers of the main loop (the compiler would otherwise hold or spill them there)
__device__ __forceinline__ int fresh_tid() {
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    return t;
}

static constexpr int kAnaRows = 128;  // values of l per analysis tile
// Columns per workgroup tile: 64 NCT (NCT column tiles of 32 per wave, two waves across).
// Launches with at most 64 active columns (up to 32 maps) take NCT = 1, so that no wave
// computes columns past the batch; every output column sees the same sequence of matrix
// operations with either tile, so results do not depend on the tile.
__host__ __device__ constexpr int col_tile(int nct) { return 64 * nct; }
// LDS floats of a kernel: its main-loop tiles or the epilogue staging (4 waves x 64 rows x
// 36), whichever is larger
__host__ __device__ constexpr int lds_floats(int main_floats) {
    return main_floats > 4 * 64 * 36 ? main_floats : 4 * 64 * 36;
}

// analysis: tile = (m, 128 values of l, 64 NCT columns); K loop over chunks of 32 ring
// pairs.  Wave w: rows 64 (w & 1) .. +63 of the tile (32 even, 32 odd l + m), columns
// 32 NCT (w >> 1) .. +32 NCT - 1.  Output: raw sums a (if a_out) and/or the Wiener-filtered coefficients
// s = scale_s C_l / (C_l + lto) a (if s_out), rows [alm][C2].  Even l + m rows contract
// G_N + G_S and odd rows G_N - G_S (a table with lambda's mirror symmetry); flip swaps the
// two, for a table that is odd where lambda is even (the spin-2 F-).  Waves per SIMD: 4
// for the one-tile table kernel (128 registers, the chunk sums included), 3 where lambda is
// generated (its recurrence state needs more), 2 for two column tiles.  NW = 8: eight
// waves (128 columns of one-tile waves) share each lambda tile, which a launch of more than
// 64 active columns otherwise reads once per 64-column group.
template <int NCT, bool GEN, int NW = 4>
__global__ void __launch_bounds__(64 * NW, NCT == 1 ? (GEN ? 3 : 4) : 2)
k_gemm_analysis(const float *__restrict__ lam, LamGen gen, const long *__restrict__ loff,
                const int *__restrict__ Lp, const int *__restrict__ minls32,
                const int2 *__restrict__ items, const int *__restrict__ tab, int per_xcd,
                const float *__restrict__ ph32, const long *__restrict__ mofs,
                const double *__restrict__ cl, float *__restrict__ a_out,
                float *__restrict__ s_out, double scale_s, double lto, int lmax, int npair,
                int Rp, int nring, int nm, int C2, int ncols, int ncg,
                const double *__restrict__ tau_b, double lto_per_tau, int flip) {
    static_assert(NW == 4 || (NW == 8 && NCT == 1), "eight waves only with one-tile waves");
    // threads; columns; lambda and X float4 loads per thread
    constexpr int NTH = 64 * NW, CT = col_tile(NCT) * NW / 4, NL = 1024 / NTH, NX = 8 * CT / NTH;
    // lambda tile [pair][row] and X_0, X_1 tiles [pair][col]; reused by the epilogue
    __shared__ __align__(16) float lds[lds_floats(32 * (kAnaRows + 4) + 2 * 32 * (CT + 4))];
    __shared__ double sAc[2][GEN ? kAnaRows : 1];  // A_lm, c_lm of the tile's rows (GEN)
    float (*sl)[kAnaRows + 4] = reinterpret_cast<float (*)[kAnaRows + 4]>(lds);
    float (*sx)[32][CT + 4] = reinterpret_cast<float (*)[32][CT + 4]>(lds + 32 * (kAnaRows + 4));
    const XcdTile xt = xcd_tile(tab, per_xcd, ncg);
    if (xt.item < 0) return;
    const int2 it = items[xt.item];
    const int m = it.x, t = it.y, cg = xt.cg;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lh = w & 1, ch = w >> 1;
    const int L = Lp[m];
    const int lhi = m + kAnaRows * t + kAnaRows - 1;  // last l of the tile
    const int lhi_w = m + kAnaRows * t + 64 * lh + 63;  // last l of this wave's rows
    const int nchunk = Rp / 32;
    const int *ms = minls32 + m * nchunk;
    floatx16 acc[2][NCT];  // [parity][column tile]
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < NCT; b++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[a][b][r] = 0.f;
    const float *lrow = GEN ? nullptr : lam + loff[m] + kAnaRows * t;
    const int wcol = 32 * NCT * ch;  // first column of this wave within the tile
    // a wave whose columns are past the batch or whose rows are all past lmax (the padding
    // of a tile that ends beyond lmax) does no products
    const bool wave_on = (CT * cg + wcol) < ncols && m + kAnaRows * t + 64 * lh <= lmax;
    floatx4 rl[NL], rn[NX], rs[NX];
    // GEN: thread (pair gpp = tid / 8, rows 16 (tid % 8) ..) of a chunk, threads 0..255; its
    // segment state, start index, seeds and z, loaded with the chunk's other operands
    const int gpp = threadIdx.x >> 3, gk = threadIdx.x & 7;
    const bool gen_thread = NW == 4 || threadIdx.x < 256;
    double2 gst = make_double2(0.0, 0.0), gsd = gst;
    double gz = 0.0;
    int gls = lmax + 1;
    if constexpr (GEN) {
        const long aoff = mofs[m] - m;
        if (threadIdx.x < kAnaRows) {
            const int l = min(m + kAnaRows * t + (int)threadIdx.x, lmax);
            sAc[0][threadIdx.x] = gen.A[aoff + l];
            sAc[1][threadIdx.x] = gen.c[aoff + l];
        }  // visible after the first barrier of the K loop
    }
    auto load = [&](int pc) __attribute__((always_inline)) {
        if constexpr (GEN) {
            if (gen_thread) {
                const int p = 32 * pc + gpp, pq = min(p, npair - 1);
                gst = gen.lck[(gen.segoff[m] + 8 * t + gk) * (long)Rp + p];
                gsd = gen.seed[(long)m * npair + pq];
                gz = gen.z[pq];
                gls = p < npair ? gen.lstart[(long)m * npair + pq] : lmax + 1;  // padding: zero rows
            }
        } else {
#pragma unroll
            for (int u = 0; u < NL; u++) {  // lambda: 32 pairs x 128 rows
                const int e = threadIdx.x + NTH * u, pp = e >> 5, c4 = e & 31;
                rl[u] = ld4(lrow + (long)(32 * pc + pp) * L + 4 * c4);
            }
        }
#pragma unroll
        for (int u = 0; u < NX; u++) {  // ring-Fourier: 32 pairs x CT columns
            const int e = threadIdx.x + NTH * u, pp = e / (CT / 4), c4 = e % (CT / 4);
            const int p = 32 * pc + pp, col = CT * cg + 4 * c4;
            // loads from clamped in-range addresses; values outside the problem are zeroed
            // when they are stored to LDS, so that no wait for the loads comes before the
            // matrix products of the current chunk
            const int pq = min(p, npair - 1), cq = min(col, ncols - 4);
            rn[u] = ld4(ph32 + ((long)m * nring + pq) * C2 + cq);
            rs[u] = ld4(ph32 + ((long)m * nring + (nring - 1 - pq)) * C2 + cq);
        }
    };
    auto next_active = [&](int pc) __attribute__((always_inline)) {
        while (pc < nchunk && ms[pc] > lhi) pc++;
        return pc;
    };
    int pc = next_active(0);
    if (pc < nchunk) load(pc);
    while (pc < nchunk) {
        __syncthreads();
        if constexpr (GEN) {
            if (gen_thread)
                lam_rows16(gst, gls, gsd, gz, m + kAnaRows * t + 16 * gk, lmax,
                           [&](int r) { return sAc[0][16 * gk + r]; }, [&](int r) { return sAc[1][16 * gk + r]; },
                           [&](int q, const float (&v)[4]) {
                               st4(&sl[gpp][16 * gk + 4 * q], floatx4{v[0], v[1], v[2], v[3]});
                           });
        } else {
#pragma unroll
            for (int u = 0; u < NL; u++) {
                const int e = threadIdx.x + NTH * u, pp = e >> 5, c4 = e & 31;
                st4(&sl[pp][4 * c4], rl[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < NX; u++) {
            const int e = threadIdx.x + NTH * u, pp = e / (CT / 4), c4 = e % (CT / 4);
            const int p = 32 * pc + pp, col = CT * cg + 4 * c4;
            const bool on = p < npair && col < ncols, south = on && (nring - 1 - p != p);
            const floatx4 xn = keep4(on, rn[u]), xs = keep4(south, rs[u]);
            const floatx4 ps = xn + xs, ms = xn - xs;
            st4(&sx[0][pp][4 * c4], flip ? ms : ps);
            st4(&sx[1][pp][4 * c4], flip ? ps : ms);
        }
        __syncthreads();
        const int pn = next_active(pc + 1);
        if (pn < nchunk) load(pn);
        if (wave_on && ms[pc] <= lhi_w) {
            const int i = lane & 31, kq = lane >> 5;
            // the chunk's 32 pairs summed from zero, then added to the running sums: the
            // FP32 rounding of a sum over all rings grows with the chain of additions, and
            // chunked it grows with 32 + the number of chunks instead of their product
            floatx16 part[2][NCT];
            auto step = [&](int kk, bool first) __attribute__((always_inline)) {
                const int pp = 2 * kk + kq;
                const float2 a = *reinterpret_cast<const float2 *>(&sl[pp][64 * lh + 2 * i]);
#pragma unroll
                for (int ct = 0; ct < NCT; ct++) {
                    const float b0 = sx[0][pp][wcol + 32 * ct + i], b1 = sx[1][pp][wcol + 32 * ct + i];
                    const floatx16 z = {};
                    part[0][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b0, first ? z : part[0][ct], 0, 0, 0);
                    part[1][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b1, first ? z : part[1][ct], 0, 0, 0);
                }
            };
            step(0, true);
#pragma unroll 5
            for (int kk = 1; kk < 16; kk++) step(kk, false);
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int ct = 0; ct < NCT; ct++) acc[a][ct] += part[a][ct];
        }
        pc = pn;
    }
    // Epilogue through LDS: per column tile, every wave parks its 64 rows x 32 columns
    // ([row][36]) and stores whole 128-byte row segments with 16-byte stores (with eight
    // waves, four at a time).  Its lane indices are formed anew from the thread id, so that
    // none of them holds a register through the main loop.
    const long base = mofs[m] - m;
    const int te = fresh_tid();
    const int we = te >> 6, le = te & 63, lhe = we & 1, wcole = 32 * NCT * (we >> 1);
    float (*stage)[36] = reinterpret_cast<float (*)[36]>(lds) + 64 * (we & 3);
#pragma unroll
    for (int ct = 0; ct < NCT; ct++)
#pragma unroll
    for (int rnd = 0; rnd < NW / 4; rnd++) {
        __syncthreads();
        if ((we >> 2) == rnd)
#pragma unroll
            for (int r = 0; r < 16; r++)
#pragma unroll
                for (int par = 0; par < 2; par++) stage[2 * acc_row(r, le) + par][le & 31] = acc[par][ct][r];
        __syncthreads();
        const int col = CT * cg + wcole + 32 * ct + 4 * (le & 7);
        if ((we >> 2) != rnd || CT * cg + wcole >= ncols || col >= ncols) continue;
#pragma unroll
        for (int it = 0; it < 8; it++) {
            const int row = 8 * it + (le >> 3);
            const int l = m + kAnaRows * t + 64 * lhe + row;
            if (l > lmax) continue;
            const float4 v = *reinterpret_cast<const float4 *>(&stage[row][4 * (le & 7)]);
            const long idx = (base + l) * C2 + col;
            if (a_out) *reinterpret_cast<float4 *>(a_out + idx) = v;
            if (s_out) {
                const double C = cl[l];
                // per-map tau (serving slots): columns 2b and 2b + 1 belong to map b, so the
                // four columns of this store span maps col / 2 and col / 2 + 1
                const double lt0 = tau_b ? lto_per_tau * tau_b[col >> 1] : lto;
                const double lt1 = tau_b ? lto_per_tau * tau_b[(col >> 1) + 1] : lto;
                const double f0 = C > 0.0 ? C / (C + lt0) * scale_s : 0.0;
                const double f1 = C > 0.0 ? C / (C + lt1) * scale_s : 0.0;
                *reinterpret_cast<float4 *>(s_out + idx) =
                    make_float4((float)(f0 * v.x), (float)(f0 * v.y), (float)(f1 * v.z), (float)(f1 * v.w));
            }
        }
    }
}

// synthesis: tile = (m, 64 ring pairs, 64 NCT columns); K loop over chunks of 64 values of
// l.  Wave w: pairs 32 (w & 1) .. +31 of the tile, columns 32 NCT (w >> 1) .. +32 NCT - 1.  The south ring
// gets E - O (lambda's mirror symmetry), or O - E with flip (the spin-2 F-).
template <int NCT, bool GEN>
__global__ void __launch_bounds__(256, NCT == 1 ? 4 : 2)
k_gemm_synthesis(const float *__restrict__ lam, LamGen gen, const long *__restrict__ loff,
                 const int *__restrict__ Lp, const int *__restrict__ minls32,
                 const int2 *__restrict__ items, const int *__restrict__ tab, int per_xcd,
                 const float *__restrict__ s32, const long *__restrict__ mofs,
                 float *__restrict__ ph32, int lmax, int npair, int Rp, int nring, int nm,
                 int C2, int ncols, int ncg, int flip, int comb) {
    constexpr int CT = col_tile(NCT), NV = CT / 16;  // columns; coefficient float4 loads per thread
    // lambda tile [pair][l] (odd stride: no bank conflicts) and coefficient tile [l][col];
    // reused by the epilogue
    __shared__ __align__(16) float lds[lds_floats(64 * (64 + 1) + 64 * (CT + 4))];
    float (*sl)[64 + 1] = reinterpret_cast<float (*)[64 + 1]>(lds);
    float (*ss)[CT + 4] = reinterpret_cast<float (*)[CT + 4]>(lds + 64 * (64 + 1));
    const XcdTile xt = xcd_tile(tab, per_xcd, ncg);
    if (xt.item < 0) return;
    const int2 it = items[xt.item];
    const int m = it.x, pt = it.y, cg = xt.cg;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rt = w & 1, ch = w >> 1;
    const int L = Lp[m], Lm = lmax - m + 1;
    const int nchunk32 = Rp / 32;
    const int ls_tile = min(minls32[m * nchunk32 + 2 * pt], minls32[m * nchunk32 + 2 * pt + 1]);
    const int ls_wave = minls32[m * nchunk32 + 2 * pt + rt];
    const int wcol = 32 * NCT * ch;  // first column of this wave within the tile
    const bool wave_on = (CT * cg + wcol) < ncols;
    floatx16 acc[2][NCT];  // [parity][column tile]
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < NCT; b++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[a][b][r] = 0.f;
    const float *lrow = GEN ? nullptr : lam + loff[m] + (long)(64 * pt) * L;
    const long base = mofs[m];
    floatx4 rl[4], rv[NV];
    // GEN: wave w generates rows 16 w .. 16 w + 15 of the chunk for pair 64 pt + lane; the
    // rows' coefficients are the same for the whole wave (scalar loads)
    const int gw = __builtin_amdgcn_readfirstlane(w);
    double2 gst = make_double2(0.0, 0.0), gsd = gst;
    double gz = 0.0;
    int gls = lmax + 1;
    if constexpr (GEN) {
        const int p = 64 * pt + lane, pq = min(p, npair - 1);
        gsd = gen.seed[(long)m * npair + pq];
        gz = gen.z[pq];
        gls = p < npair ? gen.lstart[(long)m * npair + pq] : lmax + 1;  // padding: zero rows
    }
    auto load = [&](int rc) __attribute__((always_inline)) {
        if constexpr (GEN) {
            gst = gen.lck[(gen.segoff[m] + 4 * rc + gw) * (long)Rp + 64 * pt + lane];
        } else {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int e = threadIdx.x + 256 * u, pp = e >> 4, c4 = e & 15;
                rl[u] = ld4(lrow + (long)pp * L + 64 * rc + 4 * c4);
            }
        }
#pragma unroll
        for (int u = 0; u < NV; u++) {  // coefficients: 64 values of l x CT columns
            const int e = threadIdx.x + 256 * u, rr = e / (CT / 4), c4 = e % (CT / 4);
            const int r = 64 * rc + rr, col = CT * cg + 4 * c4;
            // zeroed outside the problem at the LDS store (no wait before the products)
            rv[u] = ld4(s32 + (base + min(r, Lm - 1)) * C2 + min(col, ncols - 4));
        }
    };
    const int first = max(0, ls_tile - m) / 64;  // first chunk with a nonzero lambda
    const int nrc = (Lm + 63) / 64;
    if (first < nrc) load(first);
    for (int rc = first; rc < nrc; rc++) {
        __syncthreads();
        if constexpr (GEN) {
            const int l0 = m + 64 * rc + 16 * gw;
            const long aoff = mofs[m] - m;
            lam_rows16(gst, gls, gsd, gz, l0, lmax,
                       [&](int r) { return gen.A[aoff + min(l0 + r, lmax)]; },
                       [&](int r) { return gen.c[aoff + min(l0 + r, lmax)]; },
                       [&](int q, const float (&v)[4]) {
#pragma unroll
                           for (int i = 0; i < 4; i++) sl[lane][16 * gw + 4 * q + i] = v[i];
                       });
        } else {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int e = threadIdx.x + 256 * u, pp = e >> 4, c4 = e & 15;
                sl[pp][4 * c4] = rl[u].x;
                sl[pp][4 * c4 + 1] = rl[u].y;
                sl[pp][4 * c4 + 2] = rl[u].z;
                sl[pp][4 * c4 + 3] = rl[u].w;
            }
        }
#pragma unroll
        for (int u = 0; u < NV; u++) {
            const int e = threadIdx.x + 256 * u, rr = e / (CT / 4), c4 = e % (CT / 4);
            const int r = 64 * rc + rr, col = CT * cg + 4 * c4;
            st4(&ss[rr][4 * c4], keep4(r < Lm && col < ncols, rv[u]));
        }
        __syncthreads();
        if (rc + 1 < nrc) load(rc + 1);
        if (wave_on && ls_wave <= m + 64 * rc + 63) {
            const int i = lane & 31, kq = lane >> 5;
            // step s = (kk, parity): operands of step s + 1 are read from LDS before the
            // products of step s are issued
            float a[2], bv[2][NCT];
            auto rd = [&](int st, int q) __attribute__((always_inline)) {
                const int rr = 4 * (st >> 1) + 2 * kq + (st & 1);  // two same-parity l per step
                a[q] = sl[32 * rt + i][rr];
#pragma unroll
                for (int ct = 0; ct < NCT; ct++) bv[q][ct] = ss[rr][wcol + 32 * ct + i];
            };
            rd(0, 0);
#pragma unroll
            for (int st = 0; st < 32; st++) {
                const int q = st & 1;
                if (st + 1 < 32) rd(st + 1, q ^ 1);
                __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the products
#pragma unroll
                for (int ct = 0; ct < NCT; ct++)
                    acc[st & 1][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q], bv[q][ct], acc[st & 1][ct], 0, 0, 0);
            }
        }
    }
    // Epilogue through LDS: per column half, every wave parks F_N = E + O and F_S = E - O
    // of its 32 pairs x 32 columns ([2][pair][36]) and stores whole 128-byte row segments.
    // Rows are relative l = m + r, so the parity of r equals the parity of l + m.  Lane
    // indices formed anew from the thread id (no registers held through the main loop).
    const int te = fresh_tid();
    const int we = te >> 6, le = te & 63, rte = we & 1, wcole = 32 * NCT * (we >> 1);
    float (*stage)[32][36] = reinterpret_cast<float (*)[32][36]>(lds) + 2 * we;
#pragma unroll
    for (int ct = 0; ct < NCT; ct++) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const float E = acc[0][ct][r], O = acc[1][ct][r];
            stage[0][acc_row(r, le)][le & 31] = E + O;
            stage[1][acc_row(r, le)][le & 31] = flip ? O - E : E - O;
        }
        __syncthreads();
        const int col = CT * cg + wcole + 32 * ct + 4 * (le & 7);
        if (CT * cg + wcole >= ncols || col >= ncols) continue;
#pragma unroll
        for (int it = 0; it < 8; it++) {
            const int q = 8 * it + (le >> 3);  // 0..63: hemisphere q / 32, pair row q % 32
            const int hs = q >> 5, row = q & 31;
            const int p = 64 * pt + 32 * rte + row;
            if (p >= npair) continue;
            const int ring = hs ? nring - 1 - p : p;
            if (hs && ring == p) continue;  // equator: one ring
            float4 v = *reinterpret_cast<const float4 *>(&stage[hs][row][4 * (le & 7)]);
            float *o = ph32 + ((long)m * nring + ring) * C2 + col;
            if (comb) {
                // spin 2: v = R' = F- x s_EB of one map (E re, E im, B re, B im) and o holds
                // P' = F+ x s_EB: Q = -(P'_E + i R'_B), U = -(P'_B - i R'_E) over P'
                const float4 P = *reinterpret_cast<const float4 *>(o);
                v = make_float4(-P.x + v.w, -P.y - v.z, -P.z - v.y, -P.w + v.x);
            }
            *reinterpret_cast<float4 *>(o) = v;
        }
    }
}

// ---------------------------------------------------------------------------------------
// Conversions between the FP32 rows [alm][C2] and the FP64 per-map alm layout
// [map][nalm] complex, through LDS-transposed tiles.
// ---------------------------------------------------------------------------------------
// alm FP64 [nb][nalm] (complex) -> x32 [nalm][C2] FP32, times f(l) (mode: 3 copy, 2 C^-1/2)
__global__ void __launch_bounds__(256)
k_alm_to_cols(const double2 *__restrict__ alm, float *__restrict__ x32,
              const double *__restrict__ cl, const int *__restrict__ lofi, long nalm, int nb,
              int C2, int mode) {
    __shared__ float tile[64][65];  // [alm within tile][col within tile]
    const long i0 = (long)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64;  // columns c0 .. c0+63 = maps c0/2 .. c0/2+31
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
        const int ii = e & 63, bb = e >> 6;
        const long i = i0 + ii;
        const int b = c0 / 2 + bb;
        double2 v = make_double2(0.0, 0.0);
        if (i < nalm && b < nb) {
            v = alm[(long)b * nalm + i];
            if (mode == 2) {
                const double C = cl[lofi[i]];
                const double f = C > 0.0 ? 1.0 / sqrt(C) : 0.0;
                v = make_double2(f * v.x, f * v.y);
            }
        }
        tile[ii][2 * bb] = (float)v.x;
        tile[ii][2 * bb + 1] = (float)v.y;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int ii = e >> 6, cc = e & 63;
        const long i = i0 + ii;
        if (i < nalm && c0 + cc < C2) x32[i * C2 + c0 + cc] = tile[ii][cc];
    }
}

// x32 [nalm][C2] FP32 -> alm FP64 [nb][nalm], times f (mode 1: Omega; mode 3: 1)
__global__ void __launch_bounds__(256)
k_cols_to_alm(const float *__restrict__ x32, double2 *__restrict__ alm, long nalm, int nb, int C2,
              double scale) {
    __shared__ float tile[64][65];
    const long i0 = (long)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int ii = e >> 6, cc = e & 63;
        const long i = i0 + ii;
        tile[ii][cc] = (i < nalm && c0 + cc < C2) ? x32[i * C2 + c0 + cc] : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
        const int ii = e & 63, bb = e >> 6;
        const long i = i0 + ii;
        const int b = c0 / 2 + bb;
        if (i < nalm && b < nb)
            alm[(long)b * nalm + i] = make_double2(scale * tile[ii][2 * bb], scale * tile[ii][2 * bb + 1]);
    }
}

// ---------------------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------------------
int launch_lam_table(const Plan &p) {
    hipLaunchKernelGGL(k_lam_table, dim3(p.Rp / 64, p.nm), dim3(64), 0, p.stream, p.d_A, p.d_c,
                       p.d_mofs, p.d_lstart, p.d_seed, p.d_z, p.d_loff, p.d_Lp, p.d_lam, p.lmax,
                       p.npair);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_lam_ckpt(const Plan &p) {
    hipLaunchKernelGGL(k_lam_ckpt, dim3(p.Rp / 64, p.nm), dim3(64), 0, p.stream, p.d_A, p.d_mofs,
                       p.d_lstart, p.d_seed, p.d_z, p.d_Lp, p.d_segoff, p.d_lck, p.lmax, p.npair,
                       p.Rp);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_rows_to_cols(const Plan &p, int nb) {
    hipLaunchKernelGGL(k_rows_to_cols, dim3(p.nring, (p.nm + 63) / 64, (p.Bp + 63) / 64), dim3(256), 0,
                       p.stream, p.d_phf, p.d_ph32, p.nring, p.nm, p.nm32, nb, p.Bp, p.C2);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_zero_map_cols(const Plan &p, int b) {
    const long nrows = (long)p.nm * p.nring;
    hipLaunchKernelGGL(k_zero_map_cols, dim3((unsigned)std::min<long>((nrows + 255) / 256, 4096)), dim3(256),
                       0, p.stream, p.d_ph32, nrows, p.C2, b);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_cols_to_rows(const Plan &p, int nb) {
    hipLaunchKernelGGL(k_cols_to_rows, dim3(p.nring, (p.nm + 63) / 64, (nb + 63) / 64), dim3(256), 0,
                       p.stream, p.d_ph32, p.d_phf, p.nring, p.nm, p.nm32, nb, p.C2);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

// active columns of a launch: the real columns of nb maps (per map w floats) rounded up to
// whole 32-column MFMA tiles; never beyond the padded width (w Bp, a multiple of 32)
static int active_cols(int nb, int w) { return 32 * ((w * nb + 31) / 32); }

static LamGen lam_gen(const Plan &p) {
    return LamGen{p.d_lck, p.d_segoff, p.d_lstart, p.d_seed, p.d_z, p.d_A, p.d_c};
}

// table == nullptr: lambda rows generated in the kernels (the plan's segment states)
static int analysis_launch(const Plan &p, int nc, int C2, const float *table, const float *cols,
                           float *a_out, float *s_out, double scale_s, double lto,
                           const double *tau_b, double lto_per_tau, int flip) {
    // column tile choice 1: 64 columns (4 waves), 2: 128 columns (4 waves of two tiles), 3:
    // 128 columns (8 waves of one tile); at most 64 active columns always take 1
    const int choice = nc <= 64 ? 1 : p.gemm_ct[0];
    const int nct = choice == 2 ? 2 : 1, nw = choice == 3 ? 8 : 4;
    const int ct = col_tile(nct) * nw / 4, ncg = (nc + ct - 1) / ct;
    const dim3 grid(8 * p.ana_per_xcd * ncg), block(64 * nw);
    const LamGen g = lam_gen(p);
#define MFWF_ANA(NCT, GEN, NW)                                                                     \
    hipLaunchKernelGGL((k_gemm_analysis<NCT, GEN, NW>), grid, block, 0, p.stream, table, g, p.d_loff, \
                       p.d_Lp, p.d_minls32, p.d_ana_items, p.d_ana_tab, p.ana_per_xcd, cols,         \
                       p.d_mofs, p.d_cl, a_out, s_out, scale_s, lto, p.lmax, p.npair, p.Rp,          \
                       p.nring, p.nm, C2, nc, ncg, tau_b, lto_per_tau, flip)
    if (table == nullptr) {
        if (!p.d_lck) return fail(MFWF_EINVAL, "no lambda segment states in this plan");
        if (nw == 8) MFWF_ANA(1, true, 8);
        else if (nct == 1) MFWF_ANA(1, true, 4);
        else MFWF_ANA(2, true, 4);
    } else {
        if (nw == 8) MFWF_ANA(1, false, 8);
        else if (nct == 1) MFWF_ANA(1, false, 4);
        else MFWF_ANA(2, false, 4);
    }
#undef MFWF_ANA
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

static int synthesis_launch(const Plan &p, int nc, int C2, const float *table, const float *s_in,
                            float *out, int flip, int comb) {
    const int nct = (nc <= 64 || p.gemm_ct[1] == 1) ? 1 : 2, ncg = (nc + col_tile(nct) - 1) / col_tile(nct);
    const dim3 grid(8 * p.syn_per_xcd * ncg), block(256);
    const LamGen g = lam_gen(p);
#define MFWF_SYN(NCT, GEN)                                                                          \
    hipLaunchKernelGGL((k_gemm_synthesis<NCT, GEN>), grid, block, 0, p.stream, table, g, p.d_loff,   \
                       p.d_Lp, p.d_minls32, p.d_syn_items, p.d_syn_tab, p.syn_per_xcd, s_in,          \
                       p.d_mofs, out, p.lmax, p.npair, p.Rp, p.nring, p.nm, C2, nc, ncg, flip, comb)
    if (table == nullptr) {
        if (!p.d_lck) return fail(MFWF_EINVAL, "no lambda segment states in this plan");
        if (nct == 1) MFWF_SYN(1, true);
        else MFWF_SYN(2, true);
    } else {
        if (nct == 1) MFWF_SYN(1, false);
        else MFWF_SYN(2, false);
    }
#undef MFWF_SYN
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_gemm_analysis(const Plan &p, int nb, float *a_out, float *s_out, double scale_s,
                         double lto, double lto_per_tau) {
    return analysis_launch(p, active_cols(nb, 2), p.C2, p.lam_gen ? nullptr : p.d_lam, p.d_ph32,
                           a_out, s_out, scale_s,
                           lto, s_out ? p.d_tau : nullptr, lto_per_tau, 0);
}

int launch_gemm_synthesis(const Plan &p, int nb) {
    return synthesis_launch(p, active_cols(nb, 2), p.C2, p.lam_gen ? nullptr : p.d_lam, p.d_s32,
                            p.d_ph32, 0, 0);
}

// Raw analysis sums a_out[alm][w Bp] = table x cols[m][ring][w Bp] for nb maps of w columns
int launch_gemm_analysis_raw(const Plan &p, int nb, int w, const float *table, const float *cols,
                             float *a_out, int flip) {
    return analysis_launch(p, active_cols(nb, w), w * p.Bp, table, cols, a_out, nullptr, 0.0, 0.0,
                           nullptr, 0.0, flip);
}

// Synthesis out[m][ring][w Bp] = table x s_in[alm][w Bp] for nb maps of w columns; comb
// (w = 4): out holds P' and receives (Q, U) formed from it and this product R'
int launch_gemm_synthesis_on(const Plan &p, int nb, int w, const float *table, const float *s_in,
                             float *out, int flip, int comb) {
    if (comb && w != 4) return fail(MFWF_EINVAL, "combined synthesis needs four columns per map");
    return synthesis_launch(p, active_cols(nb, w), w * p.Bp, table, s_in, out, flip, comb);
}

int launch_alm_to_cols(const Plan &p, const double2 *alm, float *x32, int nb, int mode) {
    hipLaunchKernelGGL(k_alm_to_cols, dim3((p.nalm + 63) / 64, (p.C2 + 63) / 64), dim3(256), 0,
                       p.stream, alm, x32, p.d_cl, p.d_lofi, p.nalm, nb, p.C2, mode);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

int launch_cols_to_alm(const Plan &p, const float *x32, double2 *alm, int nb, double scale) {
    hipLaunchKernelGGL(k_cols_to_alm, dim3((p.nalm + 63) / 64, (p.C2 + 63) / 64), dim3(256), 0,
                       p.stream, x32, alm, p.nalm, nb, p.C2, scale);
    MFWF_HIP(hipGetLastError());
    return MFWF_OK;
}

}  // namespace mfwf
