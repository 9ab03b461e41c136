// Front-to-back alpha compositing, forward and backward (gfx950).
//
// Paper Section 4: the rasterisation operator renders one camera (or a tile
// of it) after the depth sort, and its backward accumulates gradients into
// the Gaussians with atomics.  The compositing rule is that of 3D Gaussian
// Splatting: per pixel, over its tile's depth-sorted list,
//   alpha = min(0.99, sigma * exp(-d^T Q d / 2)), skip alpha < 1/255,
//   stop before T would drop below 1e-4, C += alpha T c, T *= 1 - alpha.
//
// GPU organisation.  A work unit is one wavefront on a BW x BH block of a
// tile; lane l owns P horizontally adjacent pixels of one row.  The wave walks
// its tile's list in batches of 64 entries: lane l gathers entry k0 + l (its
// splat index, then its 48-byte record) with vector loads, so a batch puts 64
// independent gathers in flight, and the next batch is requested before the
// current one is composited.  Each record carries a conservative pixel box of
// its alpha >= 1/255 region; every lane tests its own entry against the
// wave's block and a ballot leaves the entries that can touch it, which
// cannot change any result since every pixel outside the box would have
// skipped the entry anyway.  The batch is copied to a wave-private LDS stage
// and the wave composites the surviving entries in list order, reading each
// record back with broadcast LDS loads (two fields by readlane in the
// forward) so that the per-pixel arithmetic takes it as uniform operands
// without spending vector issue slots on readlanes.  Waves of a tile
// never synchronise; each stops as soon as all of its pixels have terminated
// (ballot).  The backward walks the same list from the back in the same
// batches, recovers T before each entry by dividing by (1 - alpha), and
// pre-reduces the nine per-Gaussian gradient values across the wave with DPP
// before nine lanes issue one float atomic.
#include "gs_device.h"

namespace gs {
namespace {

// One list entry per lane: the 48-byte record of its splat, fetched with
// vector loads so that a whole batch of gathers is in flight at once.
struct Rec {
    float4 a, b, c;   // u, v, m00, m10 | m11, log2 sigma, r, g | b, sigma, box x, box y
};

// A wave's copy of its current batch in LDS (the backward reads each record
// back with three broadcast LDS loads instead of eleven readlanes, which
// would take VALU issue slots from the per-pixel work that bounds it).
struct WaveStage {
    float4 rec[3][GS_WAVE];   // rec[2] holds (b, splat index, 1 / sigma, -): the box is only needed by the cull
};

// A wave's copy of part of its current batch in LDS: the forward reads an
// entry's (u, v, m00, m10) and its colour with broadcast LDS loads instead
// of seven readlanes, which take vector issue slots from the per-pixel work
// that bounds it (m11 and log2 sigma stay on readlanes, so that the LDS
// return path is not the limit).
struct ColStage {
    float4 a[GS_WAVE];
    float4 col[GS_WAVE];
};

__device__ __forceinline__ Rec load_rec(const float* __restrict__ base, int gid)
{
    const float4* p = reinterpret_cast<const float4*>(base + (size_t)gid * GS_SPLAT_FLOATS);
    return Rec{p[0], p[1], p[2]};
}

// does the packed [lo, hi] int16 range miss [b0, b1]?
__device__ __forceinline__ bool misses(int packed, int b0, int b1)
{
    const int lo = (int)(short)(packed & 0xFFFF);
    const int hi = packed >> 16;
    return hi < b0 || lo > b1;
}

__device__ __forceinline__ float sq(float x) { return x * x; }

__device__ __forceinline__ float lane_f(float x, int j)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
}

// Can the splat of record e reach alpha >= 1/255 at any pixel centre of the
// block [bx0, bx1] x [by0, by1]?  A pixel at offset d = (u, v) - centre gets
// alpha = sigma 2^-q' with q' = w0^2 + w1^2, w0 = m00 dx + m10 dy, w1 = m11 dy
// (the record's factor of the scaled conic), so it is reached only where
// q' <= log2(255 sigma).  q' is convex, so its minimum over the rectangle of
// pixel centres is 0 when the rectangle holds d = 0 and otherwise lies on an
// edge, where it is a one-dimensional quadratic minimised in closed form.
// The threshold is widened by 0.02 (in log2 units) so that float32 rounding
// here and in the per-pixel alpha cannot drop a pixel the alpha test keeps;
// a wave skipping an entry that fails this test changes no result bit.
__device__ __forceinline__ bool block_may_take(const Rec& e, int bx0, int bx1, int by0, int by1)
{
    const float m00 = e.a.z, m10 = e.a.w, m11 = e.b.x;
    const float X0 = e.a.x - ((float)bx1 + 0.5f), X1 = e.a.x - ((float)bx0 + 0.5f);
    const float Y0 = e.a.y - ((float)by1 + 0.5f), Y1 = e.a.y - ((float)by0 + 0.5f);
    const bool inside = X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f;
    // edges dx = X: the minimising dy is -m00 m10 X / (m10^2 + m11^2)
    const float ra = __builtin_amdgcn_rcpf(m10 * m10 + m11 * m11);
    const float dya = fminf(fmaxf(-m00 * m10 * X0 * ra, Y0), Y1);
    const float dyb = fminf(fmaxf(-m00 * m10 * X1 * ra, Y0), Y1);
    // edges dy = Y: the minimising dx is -m10 Y / m00
    const float rm = __builtin_amdgcn_rcpf(m00);
    const float dxa = fminf(fmaxf(-m10 * Y0 * rm, X0), X1);
    const float dxb = fminf(fmaxf(-m10 * Y1 * rm, X0), X1);
    const float qa = sq(m00 * X0 + m10 * dya) + sq(m11 * dya);
    const float qb = sq(m00 * X1 + m10 * dyb) + sq(m11 * dyb);
    const float qc = sq(m00 * dxa + m10 * Y0) + sq(m11 * Y0);
    const float qd = sq(m00 * dxb + m10 * Y1) + sq(m11 * Y1);
    const float qmin = fminf(fminf(qa, qb), fminf(qc, qd));
    return inside || qmin <= e.b.y + (7.99435344f + 0.02f);
}

// A wave covers a BW x BH pixel block; BW / P lanes per pixel row.
template <int TS, int BW, int P>
struct Layout {
    static constexpr int LPR = BW / P;
    static constexpr int BH = GS_WAVE / LPR;
    static constexpr int WX = TS / BW;          // blocks per tile row
    static constexpr int WPT = WX * (TS / BH);  // waves per tile
    static_assert(BW % P == 0 && GS_WAVE % LPR == 0 && TS % BW == 0 && TS % BH == 0, "bad layout");
};

struct Unit {
    int v;               // view
    int px0, py;         // this lane's first pixel
    int bx0, by0;        // block origin (uniform)
};

template <int TS, int BW, int P>
__device__ __forceinline__ Unit unit_of(const ViewTable& vt, int gt, int wit)
{
    using L = Layout<TS, BW, P>;
    Unit u;
    u.v = view_of_tile(vt, gt);
    const int lt = gt - vt.tile_off[u.v];
    const int TX = vt.tiles_x[u.v];
    const int ty = lt / TX, tx = lt - ty * TX;
    u.bx0 = tx * TS + (wit % L::WX) * BW;
    u.by0 = ty * TS + (wit / L::WX) * L::BH;
    const int lane = __lane_id();
    u.px0 = u.bx0 + (lane % L::LPR) * P;
    u.py = u.by0 + lane / L::LPR;
    return u;
}

template <int TS, int BW, int P, bool COUNT>
__device__ __forceinline__ void fwd_unit(const ViewTable& vt, int gt, int wit,
                                         const float* __restrict__ splats,
                                         const int* __restrict__ gids,
                                         const int2* __restrict__ ranges, long long N, float bg0,
                                         float bg1, float bg2, float* __restrict__ img,
                                         float* __restrict__ Tout, int* __restrict__ lastout,
                                         int* __restrict__ visits, ColStage* __restrict__ cst)
{
    using L = Layout<TS, BW, P>;
    const Unit U = unit_of<TS, BW, P>(vt, gt, wit);
    const int W = vt.W[U.v], H = vt.H[U.v];
    const int bx1 = U.bx0 + BW - 1, by1 = U.by0 + L::BH - 1;
    const float fy = (float)U.py + 0.5f;
    float fx[P], T[P], C0[P], C1[P], C2[P];
    int last[P], stopk[P];
    // live[p]: wave-uniform mask of the lanes whose pixel p is still
    // compositing.  Kept as a scalar bit mask (not a per-lane flag) so that
    // every vote below is one compare and scalar mask arithmetic.
    uint64_t live[P];
#pragma unroll
    for (int p = 0; p < P; p++) {
        fx[p] = (float)(U.px0 + p) + 0.5f;
        T[p] = 1.0f;
        C0[p] = C1[p] = C2[p] = 0.0f;
        last[p] = 0;
        stopk[p] = -1;
        live[p] = __ballot(U.px0 + p < W && U.py < H);
    }
    const int2 r = ranges[gt];
    const float* base = splats + (size_t)U.v * (size_t)N * GS_SPLAT_FLOATS;
    const int lane = __lane_id();
    // batches of GS_WAVE list entries, one per lane.  Loads run ahead: while
    // batch b is composited, the records of batch b + 1 and the splat indices
    // of batch b + 2 are in flight.  Indices past the list end are clamped to
    // its last entry, so every load is unconditional and in bounds.
    if (r.y > r.x) {
        const int kl = r.y - 1;
        int g_nxt = gids[min(r.x + GS_WAVE + lane, kl)];
        Rec cur = load_rec(base, gids[min(r.x + lane, kl)]);
        bool alive = true;
        for (int kb = r.x; alive && kb < r.y; kb += GS_WAVE) {
            const Rec nxt = load_rec(base, g_nxt);
            const int g_nn = gids[min(kb + 2 * GS_WAVE + lane, kl)];
            // lane-parallel cull: entries whose alpha box misses this wave's
            // block cannot change any of its pixels
            const bool hit = kb + lane < r.y && !misses(__float_as_int(cur.c.z), U.bx0, bx1) &&
                             !misses(__float_as_int(cur.c.w), U.by0, by1) &&
                             block_may_take(cur, U.bx0, bx1, U.by0, by1);
            unsigned long long mask = __ballot(hit);
            // lanes read each other's stage slots: the wave barriers order
            // the previous batch's reads before these writes and the writes
            // before this batch's reads (they emit no instruction; LDS
            // operations of one wave complete in issue order)
            __builtin_amdgcn_wave_barrier();
            cst->a[lane] = cur.a;
            cst->col[lane] = make_float4(cur.b.z, cur.b.w, cur.c.x, 0.0f);
            __builtin_amdgcn_wave_barrier();
            while (mask) {
                uint64_t any_live = 0;
#pragma unroll
                for (int p = 0; p < P; p++) any_live |= live[p];
                if (any_live == 0ull) {
                    alive = false;
                    break;
                }
                const int j = __builtin_ctzll(mask);
                mask &= mask - 1;
                const float4 ea = cst->a[j];
                // the colour is read with the geometry, so a taken entry waits
                // for one LDS round trip, not two
                const float4 cc = cst->col[j];
                const float su = ea.x, sv = ea.y, m00 = ea.z, m10 = ea.w;
                const float m11 = lane_f(cur.b.x, j), ls = lane_f(cur.b.y, j);
                const float dy = sv - fy;
                const int k1 = kb + j - r.x + 1;
                // alpha first: an entry no live pixel of the wave takes costs no more
                float alp[P];
                uint64_t take[P], any_take = 0;
#pragma unroll
                for (int p = 0; p < P; p++) {
                    alp[p] = fminf(falloff(su - fx[p], dy, m00, m10, m11, ls).araw, kAlphaMax);
                    take[p] = __ballot(alp[p] >= kAlphaMin) & live[p];
                    any_take |= take[p];
                }
                // keeps the colour load above the branch (it would otherwise be
                // sunk into the taken path and issued only there)
                asm volatile("" ::"v"(cc.x), "v"(cc.y), "v"(cc.z));
                if (any_take == 0ull) continue;
                const float cr = cc.x, cg = cc.y, cb = cc.z;
#pragma unroll
                for (int p = 0; p < P; p++) {
                    const float al = alp[p];
                    const float Tn = __builtin_fmaf(-T[p], al, T[p]);
                    // a pixel stops before the entry that would take T below 1e-4
                    const uint64_t stop = __ballot(Tn < kTMin) & take[p];
                    live[p] &= ~stop;
                    if (COUNT) stopk[p] = __builtin_amdgcn_inverse_ballot_w64(stop) ? k1 : stopk[p];
                    const bool ok = __builtin_amdgcn_inverse_ballot_w64(take[p] & ~stop);
                    const float wgt = ok ? al * T[p] : 0.0f;
                    C0[p] = __builtin_fmaf(wgt, cr, C0[p]);
                    C1[p] = __builtin_fmaf(wgt, cg, C1[p]);
                    C2[p] = __builtin_fmaf(wgt, cb, C2[p]);
                    T[p] = ok ? Tn : T[p];
                    last[p] = ok ? k1 : last[p];
                }
            }
            cur = nxt;
            g_nxt = g_nn;
        }
    }
    const long long po = U.v < 0 ? 0 : vt.pix_off[U.v];
    const long long plane = (long long)W * H;
#pragma unroll
    for (int p = 0; p < P; p++) {
        if (U.px0 + p < W && U.py < H) {
            const long long pix = (long long)U.py * W + U.px0 + p;
            img[3 * po + pix] = __builtin_fmaf(T[p], bg0, C0[p]);
            img[3 * po + plane + pix] = __builtin_fmaf(T[p], bg1, C1[p]);
            img[3 * po + 2 * plane + pix] = __builtin_fmaf(T[p], bg2, C2[p]);
            Tout[po + pix] = T[p];
            lastout[po + pix] = last[p];
            // list entries this pixel examined: up to its stop, else the whole list
            if (COUNT) visits[po + pix] = stopk[p] >= 0 ? stopk[p] : r.y - r.x;
        }
    }
}

// L2: the upstream image gradient is that of the L2 loss, formed here from
// the image and the target (dimg then holds the image) as the loss kernel
// forms it, 2 (img - target) / n; the wave's share of the loss sum (float
// over its pixels, like the loss kernel's per-thread sums) goes to
// part[tile * waves per tile + wave].
template <int TS, int BW, int P, bool HAS_DA, bool L2 = false>
__device__ __forceinline__ void bwd_unit(const ViewTable& vt, int gt, int wit,
                                         const float* __restrict__ splats,
                                         const int* __restrict__ gids,
                                         const int2* __restrict__ ranges, long long N, float bg0,
                                         float bg1, float bg2, const float* __restrict__ Tfin,
                                         const int* __restrict__ nlast,
                                         const float* __restrict__ dimg,
                                         const float* __restrict__ dalpha,
                                         float* __restrict__ grad2d, WaveStage* __restrict__ stage,
                                         const float* __restrict__ tgt = nullptr, float l2scale = 0.0f,
                                         double* __restrict__ part = nullptr)
{
    using L = Layout<TS, BW, P>;
    const Unit U = unit_of<TS, BW, P>(vt, gt, wit);
    const int W = vt.W[U.v], H = vt.H[U.v];
    const int bx1 = U.bx0 + BW - 1, by1 = U.by0 + L::BH - 1;
    const long long po = vt.pix_off[U.v];
    const long long plane = (long long)W * H;
    const float fy = (float)U.py + 0.5f;
    float fx[P], T[P], S0[P], S1[P], S2[P], g0[P], g1[P], g2[P], gA[P];
    int last[P];
    int kmax = 0;
    float lsum = 0.0f;
    // The pixel inputs are loaded unconditionally, so that all of them are in
    // flight at once (a load guarded by the pixel test becomes a branch with
    // a wait of its own, one memory round trip per plane); a pixel outside
    // the view reads the view's first pixel and is then masked.
    bool in[P];
    float tv[P], a0v[P], a1v[P], a2v[P], b0v[P], b1v[P], b2v[P], dav[P];
    int lv[P];
#pragma unroll
    for (int p = 0; p < P; p++) {
        in[p] = U.px0 + p < W && U.py < H;
        const long long pix = in[p] ? (long long)U.py * W + U.px0 + p : 0;
        tv[p] = Tfin[po + pix];
        lv[p] = nlast[po + pix];
        a0v[p] = dimg[3 * po + pix];
        a1v[p] = dimg[3 * po + plane + pix];
        a2v[p] = dimg[3 * po + 2 * plane + pix];
        b0v[p] = L2 ? tgt[3 * po + pix] : 0.0f;
        b1v[p] = L2 ? tgt[3 * po + plane + pix] : 0.0f;
        b2v[p] = L2 ? tgt[3 * po + 2 * plane + pix] : 0.0f;
        dav[p] = HAS_DA ? dalpha[po + pix] : 0.0f;
    }
#pragma unroll
    for (int p = 0; p < P; p++) {
        fx[p] = (float)(U.px0 + p) + 0.5f;
        T[p] = in[p] ? tv[p] : 1.0f;
        last[p] = in[p] ? lv[p] : 0;
        if (L2) {
            const float e0 = in[p] ? a0v[p] - b0v[p] : 0.0f;
            const float e1 = in[p] ? a1v[p] - b1v[p] : 0.0f;
            const float e2 = in[p] ? a2v[p] - b2v[p] : 0.0f;
            g0[p] = l2scale * e0;
            g1[p] = l2scale * e1;
            g2[p] = l2scale * e2;
            lsum = __builtin_fmaf(e0, e0, lsum);
            lsum = __builtin_fmaf(e1, e1, lsum);
            lsum = __builtin_fmaf(e2, e2, lsum);
        } else {
            g0[p] = in[p] ? a0v[p] : 0.0f;
            g1[p] = in[p] ? a1v[p] : 0.0f;
            g2[p] = in[p] ? a2v[p] : 0.0f;
        }
        // d(1 - T_N)/d alpha_k = T_N / (1 - alpha_k): keep gA * T_N
        gA[p] = (HAS_DA && in[p]) ? dav[p] * T[p] : 0.0f;
        S0[p] = bg0;
        S1[p] = bg1;
        S2[p] = bg2;
        kmax = max(kmax, last[p]);
    }
    if (L2) {
        const float ws = wave_sum(lsum);
        if (__lane_id() == 0) part[(size_t)gt * L::WPT + wit] = (double)ws;
    }
    // the wave maximum is uniform; readfirstlane lets the compiler know, so the
    // batch loop's control stays scalar
    kmax = __builtin_amdgcn_readfirstlane(wave_max_i(kmax));
    const int2 r = ranges[gt];
    kmax = min(kmax, r.y - r.x);
    const float* base = splats + (size_t)U.v * (size_t)N * GS_SPLAT_FLOATS;
    float* gbase = grad2d + (size_t)U.v * (size_t)N * GS_GRAD_FLOATS;
    const int lane = __lane_id();
    // factor of the gradient value this lane's wave sum carries: the q'
    // derivatives (slots 0-4) leave out -ln 2 and, per slot, 2, 2, c0, 2 c0, c0
    const int jl = wave_sum9_slot(lane);
    const float gscale =
        jl < 2 ? -2.0f * kLn2 : (jl == 3 ? -2.0f * kC0 * kLn2 : (jl == 2 || jl == 4 ? -kC0 * kLn2 : 1.0f));
    // batches walk the list from its last contributing entry backwards: lane
    // l of the batch starting at kb holds entry kb - l.  As in the forward,
    // the next batch's records and the one after's indices are in flight
    // while a batch is processed; indices before the list start are clamped.
    if (kmax > 0) {
        const int kend = r.x + kmax - 1;
        int g_cur = gids[max(kend - lane, r.x)];
        int g_nxt = gids[max(kend - GS_WAVE - lane, r.x)];
        Rec cur = load_rec(base, g_cur);
        for (int kb = kend; kb >= r.x; kb -= GS_WAVE) {
            const Rec nxt = load_rec(base, g_nxt);
            const int g_nn = gids[max(kb - 2 * GS_WAVE - lane, r.x)];
            const bool hit = kb - lane >= r.x && !misses(__float_as_int(cur.c.z), U.bx0, bx1) &&
                             !misses(__float_as_int(cur.c.w), U.by0, by1) &&
                             block_may_take(cur, U.bx0, bx1, U.by0, by1);
            unsigned long long mask = __ballot(hit);
            // cross-lane stage exchange, ordered by wave barriers as in the forward
            __builtin_amdgcn_wave_barrier();
            stage->rec[0][lane] = cur.a;
            stage->rec[1][lane] = cur.b;
            // 1 / sigma once per staged entry, not once per composited entry
            stage->rec[2][lane] =
                make_float4(cur.c.x, __int_as_float(g_cur), __builtin_amdgcn_rcpf(cur.c.y), 0.0f);
            __builtin_amdgcn_wave_barrier();
            while (mask) {
                const int j = __builtin_ctzll(mask);
                mask &= mask - 1;
                const float4 ra = stage->rec[0][j];
                const float4 rb = stage->rec[1][j];
                // colour, opacity and index are read with the geometry: one LDS
                // round trip per composited entry instead of two
                const float4 rc = stage->rec[2][j];
                const float su = ra.x, sv = ra.y, m00 = ra.z, m10 = ra.w, m11 = rb.x, ls = rb.y;
                const float dy = sv - fy;
                const int kk = kb - j - r.x;
                // alpha first: an entry no pixel of the wave composited costs no more
                Falloff fp[P];
                bool okp[P], any = false;
#pragma unroll
                for (int p = 0; p < P; p++) {
                    fp[p] = falloff(su - fx[p], dy, m00, m10, m11, ls);
                    okp[p] = kk < last[p] && fminf(fp[p].araw, kAlphaMax) >= kAlphaMin;
                    any = any || okp[p];
                }
                // keeps those loads above the branch
                asm volatile("" ::"v"(rb.z), "v"(rb.w), "v"(rc.x), "v"(rc.y), "v"(rc.z));
                if (__ballot(any) == 0ull) continue;
                const int gid = __builtin_amdgcn_readfirstlane(__float_as_int(rc.y));
                const float cr = rb.z, cg = rb.w, cb = rc.x;
                const float inv_sig = rc.z;
                // a0..a4 leave out constant factors (-ln 2 times 2, 2, c0,
                // 2 c0, c0) that are applied once to the wave sums (gscale)
                float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f, a5 = 0.f, a6 = 0.f, a7 = 0.f, a8 = 0.f;
#pragma unroll
                for (int p = 0; p < P; p++) {
                    const float dx = su - fx[p];
                    const Falloff f = fp[p];
                    const float al = fminf(f.araw, kAlphaMax);
                    const bool ok = okp[p];
                    // an entry a pixel skipped contributes nothing and changes
                    // nothing: zero its alpha and upstream terms once instead
                    // of selecting every accumulated product
                    const float alo = ok ? al : 0.0f;
                    const float rom = __builtin_amdgcn_rcpf(1.0f - alo);
                    const float Tk = T[p] * rom;
                    const float wgt = alo * Tk;
                    const float d0 = cr - S0[p], d1 = cg - S1[p], d2 = cb - S2[p];
                    float ga = Tk * (d0 * g0[p] + d1 * g1[p] + d2 * g2[p]);
                    if (HAS_DA) ga = __builtin_fmaf(gA[p], rom, ga);
                    // d alpha / d(sigma, q') vanish where alpha is clamped at 0.99
                    const float gu = (ok && f.araw < kAlphaMax) ? ga : 0.0f;
                    // dL/dq' = -ln 2 al gu; the -ln 2 is one of the factors in gscale
                    const float gq = al * gu;
                    a6 = __builtin_fmaf(wgt, g0[p], a6);
                    a7 = __builtin_fmaf(wgt, g1[p], a7);
                    a8 = __builtin_fmaf(wgt, g2[p], a8);
                    a5 = __builtin_fmaf(f.araw * inv_sig, gu, a5);
                    // q' = |M^T d|^2:  dq'/du = 2 (M w)_x, dq'/dv = 2 (M w)_y;
                    // q' = c0 (A dx^2 + 2 B dx dy + C dy^2)
                    a0 = __builtin_fmaf(gq, m00 * f.w0, a0);
                    a1 = __builtin_fmaf(gq, __builtin_fmaf(m10, f.w0, m11 * f.w1), a1);
                    const float gqx = gq * dx;
                    a2 = __builtin_fmaf(gqx, dx, a2);
                    a3 = __builtin_fmaf(gqx, dy, a3);
                    a4 = __builtin_fmaf(gq * dy, dy, a4);
                    S0[p] = __builtin_fmaf(alo, d0, S0[p]);
                    S1[p] = __builtin_fmaf(alo, d1, S1[p]);
                    S2[p] = __builtin_fmaf(alo, d2, S2[p]);
                    T[p] = Tk;
                }
                const float acc[GS_GRAD_FLOATS] = {a0, a1, a2, a3, a4, a5, a6, a7, a8};
                int jj;
                const float x = wave_sum9_scatter(acc, jj) * gscale;
                if (lane < 16 && jj < GS_GRAD_FLOATS)
                    unsafeAtomicAdd(gbase + (size_t)gid * GS_GRAD_FLOATS + jj, x);
            }
            cur = nxt;
            g_cur = g_nxt;
            g_nxt = g_nn;
        }
    }
}

// Persistent waves take work in chunks of QCHUNK items from one global
// counter (one atomic per chunk keeps the counter off the critical path);
// chunk c holds items c, c + n_chunks, c + 2 n_chunks, ..., so every chunk
// mixes long and short tiles of the heavy-first order.
constexpr int QCHUNK = 8;

// claim the next chunk: lane 0 takes a ticket; the ticket is read (made
// wave-uniform) only when it is needed
__device__ __forceinline__ int claim(int* queue)
{
    int item = 0;
    if (__lane_id() == 0) item = atomicAdd(queue, 1);
    return item;
}

__device__ __forceinline__ int ticket(int pending)
{
    // keeps the read (and the wait for the atomic's return) where it is written
    asm volatile("" : "+v"(pending));
    return __builtin_amdgcn_readfirstlane(pending);
}

// tile of a grid workgroup: the workgroup index itself, or its entry in a
// dispatch order (workgroups start in index order, so the order decides which
// tiles start first and, since consecutive workgroups go to different XCDs,
// which tiles share an L2); out-of-range entries are skipped
__device__ __forceinline__ int tile_of_block(const int* __restrict__ order, int total_tiles)
{
    const int b = blockIdx.x;
    const int gt = order ? order[b] : b;
    return (unsigned)gt < (unsigned)total_tiles ? gt : -1;
}

template <int TS, int BW, int P, bool COUNT>
__global__ __launch_bounds__((GS_WAVE * Layout<TS, BW, P>::WPT)) void k_raster_fwd(
    ViewTable vt, const float* __restrict__ splats, const int* __restrict__ gids,
    const int2* __restrict__ ranges, long long N, float bg0, float bg1, float bg2,
    const int* __restrict__ order, float* __restrict__ img, float* __restrict__ Tout,
    int* __restrict__ lastout, int* __restrict__ visits)
{
    __shared__ ColStage cst[Layout<TS, BW, P>::WPT];
    const int gt = tile_of_block(order, vt.total_tiles);
    if (gt < 0) return;
    const int wit = __builtin_amdgcn_readfirstlane(threadIdx.x / GS_WAVE);
    fwd_unit<TS, BW, P, COUNT>(vt, gt, wit, splats, gids, ranges, N, bg0, bg1, bg2, img, Tout, lastout, visits,
                               &cst[wit]);
}

template <int TS, int BW, int P>
__global__ __launch_bounds__(GS_WAVE) void k_raster_fwd_persistent(
    ViewTable vt, const float* __restrict__ splats, const int* __restrict__ gids,
    const int2* __restrict__ ranges, long long N, float bg0, float bg1, float bg2,
    const int* __restrict__ order, int* __restrict__ queue, float* __restrict__ img,
    float* __restrict__ Tout, int* __restrict__ lastout)
{
    using L = Layout<TS, BW, P>;
    __shared__ ColStage cst;
    const int n_items = vt.total_tiles * L::WPT;
    const int n_chunks = (n_items + QCHUNK - 1) / QCHUNK;
    // the next chunk is claimed before the current one is processed, so the
    // queue atomic's round trip overlaps the compositing
    int c = ticket(claim(queue));
    while (c < n_chunks) {
        const int next = claim(queue);
        for (int item = c; item < n_items; item += n_chunks) {
            const int gt = order[item / L::WPT];
            if ((unsigned)gt < (unsigned)vt.total_tiles)
                fwd_unit<TS, BW, P, false>(vt, gt, item % L::WPT, splats, gids, ranges, N, bg0, bg1, bg2, img,
                                           Tout, lastout, nullptr, &cst);
        }
        c = ticket(next);
    }
}

template <int TS, int BW, int P, bool HAS_DA>
__global__ __launch_bounds__((GS_WAVE * Layout<TS, BW, P>::WPT)) void k_raster_bwd(
    ViewTable vt, const float* __restrict__ splats, const int* __restrict__ gids,
    const int2* __restrict__ ranges, long long N, float bg0, float bg1, float bg2,
    const int* __restrict__ order, const float* __restrict__ Tfin, const int* __restrict__ nlast,
    const float* __restrict__ dimg, const float* __restrict__ dalpha, float* __restrict__ grad2d)
{
    __shared__ WaveStage stage[Layout<TS, BW, P>::WPT];
    const int gt = tile_of_block(order, vt.total_tiles);
    if (gt < 0) return;
    const int wit = __builtin_amdgcn_readfirstlane(threadIdx.x / GS_WAVE);
    bwd_unit<TS, BW, P, HAS_DA>(vt, gt, wit, splats, gids, ranges, N, bg0, bg1, bg2, Tfin, nlast, dimg, dalpha,
                                grad2d, &stage[wit]);
}

// Zero parameter gradients of the groups of 64 Gaussians that no view sees
// (flags NULL: none): the part of the projection backward that needs no 2-D
// gradient,
// spread over the compositing backward's waves, whose memory traffic leaves
// most of HBM's bandwidth unused while their vector arithmetic bounds them.
struct UnseenZero {
    const uint8_t* flags;   // [n_views][N]
    float* planes[5];       // means [3][N], log-scales [3][N], quaternions [4][N], opacity [N], SH [sh_planes][N]
    int sh_planes;
};

// wave w of n zeroes, among chunks [w C / n, (w + 1) C / n) of the C groups
// of 64 Gaussians (rounded up), the groups in which no view sees any
// Gaussian: one flag load per view, then one store per plane, at a uniform
// plane address plus the lane's offset.  Groups with a seen Gaussian are
// written whole by the projection backward, so every line of a gradient
// plane is written by one kernel, in full
__device__ __forceinline__ void zero_unseen_share(const UnseenZero& z, long long N, int n_views, long long w,
                                                  long long n)
{
    const int lane = __lane_id();
    const long long n_chunks = (N + GS_WAVE - 1) / GS_WAVE;
    const long long c_lo = (w * n_chunks + n - 1) / n, c_hi = ((w + 1) * n_chunks + n - 1) / n;
    for (long long c = c_lo; c < c_hi; c++) {
        const long long c0 = c * GS_WAVE;
        const long long g = c0 + lane;
        const long long gc = g < N ? g : N - 1;
        bool seen = false;
        for (int v = 0; v < n_views; v++) seen |= (z.flags[(long long)v * N + gc] & GS_FLAG_VISIBLE) != 0;
        // a group with a seen Gaussian is left whole to the projection backward
        if (__ballot(g < N && seen) != 0ull) continue;
        if (g < N) {
            const uint32_t off = (uint32_t)lane * 4u;
            const int count[5] = {3, 3, 4, 1, z.sh_planes};
#pragma unroll
            for (int t = 0; t < 5; t++) {
                float* const base = z.planes[t] + c0;
                for (int k = 0; k < count[t]; k++)
                    nt_store(0.0f, reinterpret_cast<float*>(reinterpret_cast<char*>(base + (long long)k * N) + off));
            }
        }
    }
}

// the backward with the L2 loss's image gradient formed from images and targets
template <int TS, int BW, int P>
__global__ __launch_bounds__((GS_WAVE * Layout<TS, BW, P>::WPT)) void k_raster_bwd_l2(
    ViewTable vt, const float* __restrict__ splats, const int* __restrict__ gids,
    const int2* __restrict__ ranges, long long N, float bg0, float bg1, float bg2,
    const int* __restrict__ order, const float* __restrict__ Tfin, const int* __restrict__ nlast,
    const float* __restrict__ img, const float* __restrict__ tgt, float l2scale, double* __restrict__ part,
    float* __restrict__ grad2d, UnseenZero uz)
{
    using L = Layout<TS, BW, P>;
    __shared__ WaveStage stage[L::WPT];
    const int gt = tile_of_block(order, vt.total_tiles);
    const int wit = __builtin_amdgcn_readfirstlane(threadIdx.x / GS_WAVE);
    // the zeroing goes to the waves of the first half of the blocks (the
    // heaviest tiles in a heavy-first order), before their compositing: its
    // stores then drain while those long waves compute.  Measured at 4K
    // against the other placements: after the compositing, or spread over
    // every wave, or over the last blocks, the kernel ran longer.
    const unsigned zb = (gridDim.x + 1) / 2;
    if (uz.flags && blockIdx.x < zb)
        zero_unseen_share(uz, N, vt.n_views, (long long)blockIdx.x * L::WPT + wit, (long long)zb * L::WPT);
    if (gt >= 0)
        bwd_unit<TS, BW, P, false, true>(vt, gt, wit, splats, gids, ranges, N, bg0, bg1, bg2, Tfin, nlast, img,
                                         nullptr, grad2d, &stage[wit], tgt, l2scale, part);
}

// Sum of the per-wave partials in a fixed order: blocks of L2_SPAN
// consecutive partials (each thread's L2_ITEMS loads in flight at once, then
// a fixed tree), then one block over the block sums.
constexpr int L2_THREADS = 256;
constexpr int L2_ITEMS = 16;
constexpr long long L2_SPAN = (long long)L2_THREADS * L2_ITEMS;

__device__ __forceinline__ double block_tree_sum(double x, double* s)
{
    s[threadIdx.x] = x;
    __syncthreads();
    for (int o = L2_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    return s[0];
}

__global__ __launch_bounds__(L2_THREADS) void k_l2_parts_sum(const double* __restrict__ part, long long np,
                                                             double* __restrict__ out)
{
    __shared__ double s[L2_THREADS];
    const long long base = (long long)blockIdx.x * L2_SPAN + threadIdx.x;
    double v[L2_ITEMS];
#pragma unroll
    for (int k = 0; k < L2_ITEMS; k++) {
        const long long i = base + (long long)k * L2_THREADS;
        v[k] = i < np ? part[i] : 0.0;
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < L2_ITEMS; k++) acc += v[k];
    const double t = block_tree_sum(acc, s);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// loss = (sum of the nb block sums, strided per thread, then a fixed tree) / n
__global__ __launch_bounds__(L2_THREADS) void k_l2_parts_final(const double* __restrict__ sums, int nb,
                                                               double inv_n, float* __restrict__ loss)
{
    __shared__ double s[L2_THREADS];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += L2_THREADS) acc += sums[i];
    const double t = block_tree_sum(acc, s);
    if (threadIdx.x == 0) loss[0] = (float)(t * inv_n);
}

template <int TS, int BW, int P, bool HAS_DA>
__global__ __launch_bounds__(GS_WAVE) void k_raster_bwd_persistent(
    ViewTable vt, const float* __restrict__ splats, const int* __restrict__ gids,
    const int2* __restrict__ ranges, long long N, float bg0, float bg1, float bg2,
    const int* __restrict__ order, int* __restrict__ queue, const float* __restrict__ Tfin,
    const int* __restrict__ nlast, const float* __restrict__ dimg, const float* __restrict__ dalpha,
    float* __restrict__ grad2d)
{
    using L = Layout<TS, BW, P>;
    __shared__ WaveStage stage;
    const int n_items = vt.total_tiles * L::WPT;
    const int n_chunks = (n_items + QCHUNK - 1) / QCHUNK;
    int c = ticket(claim(queue));
    while (c < n_chunks) {
        const int next = claim(queue);
        for (int item = c; item < n_items; item += n_chunks) {
            const int gt = order[item / L::WPT];
            if ((unsigned)gt < (unsigned)vt.total_tiles)
                bwd_unit<TS, BW, P, HAS_DA>(vt, gt, item % L::WPT, splats, gids, ranges, N, bg0, bg1, bg2, Tfin,
                                            nlast, dimg, dalpha, grad2d, &stage);
        }
        c = ticket(next);
    }
}

__global__ void k_zero_queue(int* q) { q[0] = 0; }

int persistent_blocks()
{
    static int n = 0;
    if (n == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        n = cus * 32;
    }
    return n;
}

template <int TS, int BW, int P>
hipError_t fwd_cfg(const ViewTable& vt, const float* splats, const int* gids, const int2* ranges, long long N,
                   const float* bg, const int* order, int* queue, float* img, float* Tout, int* lastout,
                   int* visits, hipStream_t st)
{
    using L = Layout<TS, BW, P>;
    if (visits) {
        hipLaunchKernelGGL((k_raster_fwd<TS, BW, P, true>), dim3(vt.total_tiles), dim3(GS_WAVE * L::WPT), 0, st,
                           vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], nullptr, img, Tout, lastout, visits);
    } else if (order && queue) {
        hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(1), 0, st, queue);
        hipLaunchKernelGGL((k_raster_fwd_persistent<TS, BW, P>), dim3(persistent_blocks()), dim3(GS_WAVE), 0,
                           st, vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], order, queue, img, Tout,
                           lastout);
    } else {
        hipLaunchKernelGGL((k_raster_fwd<TS, BW, P, false>), dim3(vt.total_tiles), dim3(GS_WAVE * L::WPT), 0,
                           st, vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], order, img, Tout, lastout,
                           nullptr);
    }
    return hipGetLastError();
}

template <int TS, int BW, int P>
hipError_t bwd_cfg(const ViewTable& vt, const float* splats, const int* gids, const int2* ranges, long long N,
                   const float* bg, const int* order, int* queue, const float* Tfin, const int* nlast,
                   const float* dimg, const float* dalpha, float* grad2d, hipStream_t st)
{
    using L = Layout<TS, BW, P>;
    if (order && queue) {
        hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(1), 0, st, queue);
        if (dalpha)
            hipLaunchKernelGGL((k_raster_bwd_persistent<TS, BW, P, true>), dim3(persistent_blocks()),
                               dim3(GS_WAVE), 0, st, vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], order,
                               queue, Tfin, nlast, dimg, dalpha, grad2d);
        else
            hipLaunchKernelGGL((k_raster_bwd_persistent<TS, BW, P, false>), dim3(persistent_blocks()),
                               dim3(GS_WAVE), 0, st, vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], order,
                               queue, Tfin, nlast, dimg, dalpha, grad2d);
    } else {
        if (dalpha)
            hipLaunchKernelGGL((k_raster_bwd<TS, BW, P, true>), dim3(vt.total_tiles), dim3(GS_WAVE * L::WPT),
                               0, st, vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], order, Tfin, nlast, dimg,
                               dalpha, grad2d);
        else
            hipLaunchKernelGGL((k_raster_bwd<TS, BW, P, false>), dim3(vt.total_tiles), dim3(GS_WAVE * L::WPT),
                               0, st, vt, splats, gids, ranges, N, bg[0], bg[1], bg[2], order, Tfin, nlast, dimg,
                               dalpha, grad2d);
    }
    return hipGetLastError();
}

template <int TS, int BW, int P>
hipError_t bwd_l2_cfg(const ViewTable& vt, const float* splats, const int* gids, const int2* ranges, long long N,
                      const float* bg, const int* order, const float* Tfin, const int* nlast, const float* img,
                      const float* tgt, long long n_elems, float* loss, double* part, float* grad2d,
                      const UnseenZero& uz, hipStream_t st)
{
    using L = Layout<TS, BW, P>;
    // the same scale as the loss kernel's gradient
    const float scale = n_elems > 0 ? (float)(2.0 / (double)n_elems) : 0.0f;
    if (vt.total_tiles > 0)
        hipLaunchKernelGGL((k_raster_bwd_l2<TS, BW, P>), dim3(vt.total_tiles), dim3(GS_WAVE * L::WPT), 0, st, vt,
                           splats, gids, ranges, N, bg[0], bg[1], bg[2], order, Tfin, nlast, img, tgt, scale,
                           part, grad2d, uz);
    // the block sums follow the largest possible number of per-wave partials
    const long long np = (long long)vt.total_tiles * L::WPT;
    const long long np_max = (long long)vt.total_tiles * (TS * TS / GS_WAVE);
    const int nb = (int)((np + L2_SPAN - 1) / L2_SPAN);
    double* sums = part + np_max;
    if (nb > 0)
        hipLaunchKernelGGL(k_l2_parts_sum, dim3(nb), dim3(L2_THREADS), 0, st, (const double*)part, np, sums);
    hipLaunchKernelGGL(k_l2_parts_final, dim3(1), dim3(L2_THREADS), 0, st, (const double*)sums, nb,
                       n_elems > 0 ? 1.0 / (double)n_elems : 0.0, loss);
    return hipGetLastError();
}

}  // namespace

// Wave blocks available per tile edge (block width, pixels per lane); the
// first entry of each list is the default.
//   tile 8:  8x8 / 1
//   tile 16: 8x8 / 1, 16x4 / 1, 16x16 / 4
//   tile 32: 8x8 / 1, 16x16 / 4, 32x8 / 4
bool raster_cfg_ok(int tile, int bw, int ppl)
{
    if (bw == 0 && ppl == 0) return tile == 8 || tile == 16 || tile == 32;
    switch (tile) {
    case 8: return bw == 8 && ppl == 1;
    case 16: return (bw == 8 && ppl == 1) || (bw == 16 && (ppl == 1 || ppl == 2 || ppl == 4));
    case 32: return (bw == 8 && ppl == 1) || (bw == 16 && (ppl == 2 || ppl == 4)) || (bw == 32 && ppl == 4);
    default: return false;
    }
}

#define GS_FWD(TS, BW, P) \
    return fwd_cfg<TS, BW, P>(vt, splats, gids, ranges, N, bg, order, queue, img, Tout, lastout, visits, st)

hipError_t launch_raster_fwd(int tile, int bw, int ppl, const ViewTable& vt, const float* splats,
                             const int* gids, const int2* ranges, long long N, const float* bg,
                             const int* order, int* queue, float* img, float* Tout, int* lastout, int* visits,
                             hipStream_t st)
{
    if (vt.total_tiles == 0) return hipSuccess;
    if (bw == 0) { bw = 8; ppl = 1; }
    switch (tile) {
    case 8: GS_FWD(8, 8, 1);
    case 16:
        if (bw == 16 && ppl == 4) GS_FWD(16, 16, 4);
        if (bw == 16 && ppl == 2) GS_FWD(16, 16, 2);
        if (bw == 16) GS_FWD(16, 16, 1);
        GS_FWD(16, 8, 1);
    default:
        if (bw == 32) GS_FWD(32, 32, 4);
        if (bw == 16 && ppl == 2) GS_FWD(32, 16, 2);
        if (bw == 16) GS_FWD(32, 16, 4);
        GS_FWD(32, 8, 1);
    }
}
#undef GS_FWD

#define GS_BWD(TS, BW, P) \
    return bwd_cfg<TS, BW, P>(vt, splats, gids, ranges, N, bg, order, queue, Tfin, nlast, dimg, dalpha, grad2d, st)

hipError_t launch_raster_bwd(int tile, int bw, int ppl, const ViewTable& vt, const float* splats,
                             const int* gids, const int2* ranges, long long N, const float* bg,
                             const int* order, int* queue, const float* Tfin, const int* nlast,
                             const float* dimg, const float* dalpha, float* grad2d, hipStream_t st)
{
    if (vt.total_tiles == 0) return hipSuccess;
    if (bw == 0) { bw = 8; ppl = 1; }
    switch (tile) {
    case 8: GS_BWD(8, 8, 1);
    case 16:
        if (bw == 16 && ppl == 4) GS_BWD(16, 16, 4);
        if (bw == 16 && ppl == 2) GS_BWD(16, 16, 2);
        if (bw == 16) GS_BWD(16, 16, 1);
        GS_BWD(16, 8, 1);
    default:
        if (bw == 32) GS_BWD(32, 32, 4);
        if (bw == 16 && ppl == 2) GS_BWD(32, 16, 2);
        if (bw == 16) GS_BWD(32, 16, 4);
        GS_BWD(32, 8, 1);
    }
}
#undef GS_BWD

// one partial per wave (at most tile^2 / 64 waves per tile: every wave covers
// at least 64 pixels), then one sum per L2_SPAN partials
size_t raster_bwd_l2_workspace_size(const ViewTable& vt, int tile)
{
    const size_t np = (size_t)vt.total_tiles * (size_t)(tile * tile / GS_WAVE);
    return sizeof(double) * (np + (np + L2_SPAN - 1) / L2_SPAN);
}

#define GS_BWDL2(TS, BW, P) \
    return bwd_l2_cfg<TS, BW, P>(vt, splats, gids, ranges, N, bg, order, Tfin, nlast, img, tgt, n_elems, loss, \
                                 (double*)part, grad2d, uz, st)

hipError_t launch_raster_bwd_l2(int tile, int bw, int ppl, const ViewTable& vt, const float* splats,
                                const int* gids, const int2* ranges, long long N, const float* bg,
                                const int* order, const float* Tfin, const int* nlast, const float* img,
                                const float* tgt, long long n_elems, float* loss, void* part, float* grad2d,
                                const uint8_t* flags, int sh_degree, float* const* unseen_grads, hipStream_t st)
{
    UnseenZero uz = {};
    if (flags && unseen_grads && N > 0) {
        uz.flags = flags;
        for (int k = 0; k < 5; k++) uz.planes[k] = unseen_grads[k];
        uz.sh_planes = 3 * (sh_degree + 1) * (sh_degree + 1);
    }
    if (bw == 0) { bw = 8; ppl = 1; }
    switch (tile) {
    case 8: GS_BWDL2(8, 8, 1);
    case 16:
        if (bw == 16 && ppl == 4) GS_BWDL2(16, 16, 4);
        if (bw == 16 && ppl == 2) GS_BWDL2(16, 16, 2);
        if (bw == 16) GS_BWDL2(16, 16, 1);
        GS_BWDL2(16, 8, 1);
    default:
        if (bw == 32) GS_BWDL2(32, 32, 4);
        if (bw == 16 && ppl == 2) GS_BWDL2(32, 16, 2);
        if (bw == 16) GS_BWDL2(32, 16, 4);
        GS_BWDL2(32, 8, 1);
    }
}
#undef GS_BWDL2

}  // namespace gs
