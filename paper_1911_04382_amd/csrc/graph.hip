// Graph setup on gfx950: validation, the CSR of L_G (eq. 1), the maximum-weight
// spanning tree by Boruvka, the rooted tree by an Euler tour, and the
// heavy-light layout that the level-scheduled tree solve runs on.
#include "graph.h"

namespace grass {

namespace {

inline int grid_for(long long n, int threads = 256, int cap = 65536) {
    long long b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    return (int)std::min<long long>(b, cap);
}
#define GSTRIDE(i, n) for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

// ------------------------------------------------------------ validation
enum : unsigned { VF_RANGE = 1, VF_ORDER = 2, VF_WEIGHT = 4 };

__global__ void k_validate(long long n, long long m, const int *__restrict__ src, const int *__restrict__ dst,
                           const double *__restrict__ w, unsigned *__restrict__ flags) {
    unsigned f = 0;
    GSTRIDE(e, m) {
        int a = src[e], b = dst[e];
        if (a < 0 || b >= n || a >= b) f |= VF_RANGE;
        double x = w[e];
        if (!(x > 0.0) || !(x < INFINITY)) f |= VF_WEIGHT;
        if (e > 0) {
            int pa = src[e - 1], pb = dst[e - 1];
            if (a < pa || (a == pa && b <= pb)) f |= VF_ORDER;
        }
    }
    if (f) atomicOr(flags, f);
}

// ------------------------------------------------------------- CSR build
__global__ void k_count_deg(long long m, const int *__restrict__ src, const int *__restrict__ dst,
                            int *__restrict__ in_cnt, int *__restrict__ out_cnt) {
    GSTRIDE(e, m) {
        atomicAdd(&out_cnt[src[e]], 1);
        atomicAdd(&in_cnt[dst[e]], 1);
    }
}
__global__ void k_add2(long long n, const int *__restrict__ a, const int *__restrict__ b, int *__restrict__ c) {
    GSTRIDE(i, n) c[i] = a[i] + b[i];
}
__global__ void k_keys_dst(long long m, const int *__restrict__ dst, unsigned long long *__restrict__ keys,
                           int *__restrict__ vals) {
    GSTRIDE(e, m) {
        keys[e] = (unsigned long long)(unsigned)dst[e];
        vals[e] = (int)e;
    }
}
// Row v of the CSR = in-neighbours (src < v, ascending) then out-neighbours
// (dst > v, ascending): rows come out sorted by neighbour id, deterministically.
__global__ void k_csr_out(long long m, const int *__restrict__ src, const int *__restrict__ dst,
                          const int *__restrict__ rowptr, const int *__restrict__ in_cnt,
                          const int *__restrict__ out_first, int *__restrict__ col, int *__restrict__ ceid) {
    GSTRIDE(e, m) {
        int v = src[e];
        long long pos = (long long)rowptr[v] + in_cnt[v] + (e - out_first[v]);
        col[pos] = dst[e];
        ceid[pos] = (int)e;
    }
}
__global__ void k_csr_in(long long m, const int *__restrict__ sorted_e, const int *__restrict__ src,
                         const int *__restrict__ dst, const int *__restrict__ rowptr, const int *__restrict__ in_first,
                         int *__restrict__ col, int *__restrict__ ceid) {
    GSTRIDE(s, m) {
        int e = sorted_e[s];
        int v = dst[e];
        long long pos = (long long)rowptr[v] + (s - in_first[v]);
        col[pos] = src[e];
        ceid[pos] = e;
    }
}
template <typename T>
__global__ void k_row_finish(long long n, const int *__restrict__ rowptr, const int *__restrict__ ceid,
                             const double *__restrict__ w, T *__restrict__ cval, double *__restrict__ deg) {
    GSTRIDE(v, n) {
        double s = 0.0;
        for (int p = rowptr[v]; p < rowptr[v + 1]; p++) {
            double x = w[ceid[p]];
            cval[p] = (T)x;
            s += x;
        }
        deg[v] = s;
    }
}
template <typename T>
__global__ void k_cast_w(long long m, const double *__restrict__ w, T *__restrict__ wT) {
    GSTRIDE(e, m) wT[e] = (T)w[e];
}

// --------------------------------------------------------------- Boruvka
// Components select their best incident edge under the total order (weight
// descending, id ascending) in two exact integer steps: max of the weight's bit
// image (positive doubles order like their bits), then min edge id among edges
// of that weight. The selected edges of a round are all tree edges of the unique
// maximum spanning tree.
__global__ void k_bor_init(long long n, int *__restrict__ comp) {
    GSTRIDE(v, n) comp[v] = (int)v;
}
__global__ void k_bor_reset(long long n, unsigned long long *__restrict__ bw, int *__restrict__ be) {
    GSTRIDE(v, n) {
        bw[v] = 0ull;
        be[v] = INT_MAX;
    }
}
__global__ void k_bor_maxw(long long m, const int *__restrict__ src, const int *__restrict__ dst,
                           const double *__restrict__ w, const int *__restrict__ comp,
                           unsigned long long *__restrict__ bw) {
    GSTRIDE(e, m) {
        int cu = comp[src[e]], cv = comp[dst[e]];
        if (cu != cv) {
            unsigned long long b = (unsigned long long)__double_as_longlong(w[e]);
            atomicMax(&bw[cu], b);
            atomicMax(&bw[cv], b);
        }
    }
}
__global__ void k_bor_mine(long long m, const int *__restrict__ src, const int *__restrict__ dst,
                           const double *__restrict__ w, const int *__restrict__ comp,
                           const unsigned long long *__restrict__ bw, int *__restrict__ be) {
    GSTRIDE(e, m) {
        int cu = comp[src[e]], cv = comp[dst[e]];
        if (cu != cv) {
            unsigned long long b = (unsigned long long)__double_as_longlong(w[e]);
            if (b == bw[cu]) atomicMin(&be[cu], (int)e);
            if (b == bw[cv]) atomicMin(&be[cv], (int)e);
        }
    }
}
__global__ void k_bor_hook(long long n, const int *__restrict__ src, const int *__restrict__ dst,
                           const int *__restrict__ comp, const int *__restrict__ be, int *__restrict__ nxt,
                           uint8_t *__restrict__ tree, int *__restrict__ counter) {
    GSTRIDE(c, n) {
        int to = (int)c;
        if (comp[c] == c && be[c] != INT_MAX) {
            int e = be[c];
            int a = comp[src[e]], b = comp[dst[e]];
            to = (a == c) ? b : a;
            tree[e] = 1;
            atomicAdd(counter, 1);
        }
        nxt[c] = to;
    }
}
// mutual selections (two components choosing the same edge) form the only cycles;
// the smaller component id becomes the root of the merged component
__global__ void k_bor_break(long long n, const int *__restrict__ comp, const int *__restrict__ nxt,
                            int *__restrict__ nxt2) {
    GSTRIDE(c, n) {
        int o = nxt[c];
        int r = o;
        if (comp[c] == c && o != c && nxt[o] == c && c < o) r = (int)c;
        nxt2[c] = r;
    }
}
// find the root of each component's hook tree with path halving (writes only
// ever replace a pointer by one of its ancestors, so concurrent walks are safe)
__global__ void k_bor_find(long long n, const int *__restrict__ comp, int *__restrict__ nxt2, int *__restrict__ fin,
                           unsigned *__restrict__ devflags) {
    GSTRIDE(c, n) {
        if (comp[c] != c) continue;
        int r = (int)c;
        long long steps = 0;
        for (;;) {
            int a = ld_agent_i32(&nxt2[r]);
            if (a == r) break;
            if (++steps > n) {  // a forest walk is shorter than n: guard against a cycle
                atomicOr(devflags, DEVERR_TREE);
                break;
            }
            int b = ld_agent_i32(&nxt2[a]);
            if (a != b) st_agent_i32(&nxt2[r], b);
            r = a;
        }
        fin[c] = r;
    }
}
__global__ void k_bor_relabel(long long n, int *__restrict__ comp, const int *__restrict__ fin) {
    GSTRIDE(v, n) comp[v] = fin[comp[v]];
}

// -------------------------------------------------------- rooted tree
__global__ void k_tree_count(long long n, const int *__restrict__ rowptr, const int *__restrict__ ceid,
                             const uint8_t *__restrict__ mask, int *__restrict__ cnt) {
    GSTRIDE(v, n) {
        int c = 0;
        for (int p = rowptr[v]; p < rowptr[v + 1]; p++) c += mask[ceid[p]] == 1;
        cnt[v] = c;
    }
}
__global__ void k_tree_fill(long long n, const int *__restrict__ rowptr, const int *__restrict__ col,
                            const int *__restrict__ ceid, const uint8_t *__restrict__ mask, const int *__restrict__ tptr,
                            int *__restrict__ tcol, int *__restrict__ teid, int *__restrict__ tsrc) {
    GSTRIDE(v, n) {
        int o = tptr[v];
        for (int p = rowptr[v]; p < rowptr[v + 1]; p++)
            if (mask[ceid[p]] == 1) {
                tcol[o] = col[p];
                teid[o] = ceid[p];
                tsrc[o] = (int)v;
                o++;
            }
    }
}
// Euler tour: the successor of arc u->v is the arc after v->u in v's (cyclic) list.
__global__ void k_euler_succ(long long L, const int *__restrict__ tptr, const int *__restrict__ tcol,
                             const int *__restrict__ tsrc, int *__restrict__ twin, int *__restrict__ succ) {
    GSTRIDE(a, L) {
        int u = tsrc[a], v = tcol[a];
        int lo = tptr[v], hi = tptr[v + 1] - 1;
        while (lo < hi) {  // rows are sorted by neighbour id
            int mid = (lo + hi) >> 1;
            if (tcol[mid] < u) lo = mid + 1;
            else hi = mid;
        }
        twin[a] = lo;
        succ[a] = (lo + 1 < tptr[v + 1]) ? lo + 1 : tptr[v];
    }
}
// cut the cycle at the root: the tour starts with the root's first arc, so the arc
// whose successor is that arc ends the tour
__global__ void k_euler_cut(const int *__restrict__ tptr, const int *__restrict__ twin, int *__restrict__ succ,
                            int root) {
    int last = tptr[root + 1] - 1;
    if (last >= tptr[root]) succ[twin[last]] = -1;
}
__global__ void k_rank_init(long long L, const int *__restrict__ succ, int *__restrict__ nx, int *__restrict__ rk) {
    GSTRIDE(a, L) {
        int s = succ[a];
        nx[a] = s;
        rk[a] = s < 0 ? 0 : 1;
    }
}
// Wyllie pointer jumping: rk = number of arcs after a in the tour
__global__ void k_rank_jump(long long L, const int *__restrict__ nx, const int *__restrict__ rk,
                            int *__restrict__ nx2, int *__restrict__ rk2) {
    GSTRIDE(a, L) {
        int s = nx[a];
        if (s >= 0) {
            rk2[a] = rk[a] + rk[s];
            nx2[a] = nx[s];
        } else {
            rk2[a] = rk[a];
            nx2[a] = -1;
        }
    }
}
__global__ void k_orient(long long L, const int *__restrict__ tsrc, const int *__restrict__ tcol,
                         const int *__restrict__ teid, const int *__restrict__ twin, const int *__restrict__ rk,
                         const double *__restrict__ w, int *__restrict__ parent, double *__restrict__ pw,
                         int *__restrict__ fpos, int *__restrict__ bpos, int *__restrict__ counter) {
    GSTRIDE(a, L) {
        int t = twin[a];
        if (rk[a] > rk[t]) {  // a = u -> v comes first: a goes down the tree
            int v = tcol[a];
            parent[v] = tsrc[a];
            pw[v] = w[teid[a]];
            fpos[v] = (int)(L - 1 - rk[a]);
            bpos[v] = (int)(L - 1 - rk[t]);
            atomicAdd(counter, 1);
        }
    }
}
__global__ void k_sizes(long long n, const int *__restrict__ fpos, const int *__restrict__ bpos,
                        const int *__restrict__ parent, int *__restrict__ size) {
    GSTRIDE(v, n) size[v] = parent[v] < 0 ? (int)n : (bpos[v] - fpos[v] + 1) / 2;
}
__global__ void k_heavy(long long n, const int *__restrict__ tptr, const int *__restrict__ tcol,
                        const int *__restrict__ parent, const int *__restrict__ size, int *__restrict__ heavy) {
    GSTRIDE(u, n) {
        int best = -1, bs = -1;
        for (int a = tptr[u]; a < tptr[u + 1]; a++) {
            int v = tcol[a];
            if (parent[v] == u) {
                int s = size[v];
                if (s > bs || (s == bs && v < best)) {
                    bs = s;
                    best = v;
                }
            }
        }
        heavy[u] = best;
    }
}
__global__ void k_hl_init(long long n, const int *__restrict__ parent, const int *__restrict__ heavy,
                          int *__restrict__ anc, int *__restrict__ dist) {
    GSTRIDE(v, n) {
        int p = parent[v];
        bool cont = p >= 0 && heavy[p] == v;
        anc[v] = cont ? p : (int)v;
        dist[v] = cont ? 1 : 0;
    }
}
__global__ void k_hl_jump(long long n, const int *__restrict__ anc, const int *__restrict__ dist,
                          int *__restrict__ anc2, int *__restrict__ dist2, int *__restrict__ changed) {
    GSTRIDE(v, n) {
        int a = anc[v];
        int aa = anc[a];
        anc2[v] = aa;
        dist2[v] = dist[v] + dist[a];
        if (aa != a) *changed = 1;
    }
}
// +1 entering a light child (a path head other than the root), -1 leaving it
__global__ void k_tour_vals(long long L, const int *__restrict__ tsrc, const int *__restrict__ tcol,
                            const int *__restrict__ twin, const int *__restrict__ rk, const int *__restrict__ parent,
                            const int *__restrict__ head, int *__restrict__ tval) {
    GSTRIDE(a, L) {
        int u = tsrc[a], v = tcol[a];
        int val = 0;
        bool down = rk[a] > rk[twin[a]];
        if (down) {
            if (head[v] == v) val = 1;
        } else {
            if (head[u] == u && parent[u] == v) val = -1;
        }
        tval[L - 1 - rk[a]] = val;
    }
}
__global__ void k_light_depth(long long n, const int *__restrict__ parent, const int *__restrict__ fpos,
                              const int *__restrict__ tscan, int *__restrict__ ld) {
    GSTRIDE(v, n) ld[v] = parent[v] < 0 ? 0 : tscan[fpos[v]];
}
__global__ void k_path_len(long long n, const int *__restrict__ head, const int *__restrict__ off,
                           int *__restrict__ plen) {
    GSTRIDE(v, n) atomicMax(&plen[head[v]], off[v] + 1);
}
__global__ void k_level_stats(long long n, const int *__restrict__ head, const int *__restrict__ ld,
                              const int *__restrict__ plen, int *__restrict__ lvl_nodes, int *__restrict__ maxld,
                              int *__restrict__ is_head) {
    GSTRIDE(v, n) {
        bool h = head[v] == v;
        is_head[v] = h ? 1 : 0;
        if (h) {
            int l = ld[v];
            if (l < kMaxLevels) atomicAdd(&lvl_nodes[l], plen[v]);
            atomicMax(maxld, l);
        }
    }
}
__global__ void k_head_keys(long long n, const int *__restrict__ is_head, const int *__restrict__ hpos,
                            const int *__restrict__ ld, unsigned long long *__restrict__ keys, int *__restrict__ vals) {
    GSTRIDE(v, n) if (is_head[v]) {
        keys[hpos[v]] = (unsigned long long)ld[v];
        vals[hpos[v]] = (int)v;
    }
}
__global__ void k_gather_plen(long long nh, const int *__restrict__ heads, const int *__restrict__ plen,
                              int *__restrict__ hl) {
    GSTRIDE(i, nh) hl[i] = plen[heads[i]];
}
__global__ void k_path_base(long long nh, const int *__restrict__ heads, const int *__restrict__ cum,
                            const int *__restrict__ ld, const long long *__restrict__ lvl_pad,
                            const long long *__restrict__ lvl_unpad, int *__restrict__ pbase) {
    GSTRIDE(i, nh) {
        int h = heads[i];
        int l = ld[h];
        pbase[h] = (int)(lvl_pad[l] + (cum[i] - lvl_unpad[l]));
    }
}
template <typename T>
__global__ void k_layout(long long n, const int *__restrict__ head, const int *__restrict__ off,
                         const int *__restrict__ pbase, const int *__restrict__ heavy, const int *__restrict__ parent,
                         const double *__restrict__ pw, int *__restrict__ lp, int *__restrict__ perm,
                         uint8_t *__restrict__ flags, int *__restrict__ ptop, T *__restrict__ rpw) {
    GSTRIDE(v, n) {
        int i = pbase[head[v]] + off[v];
        lp[v] = i;
        perm[i] = (int)v;
        flags[i] = (off[v] == 0 ? SEG_TOP : 0) | (heavy[v] < 0 ? SEG_BOT : 0);
        ptop[i] = off[v] == 0 ? parent[v] : -1;
        rpw[i] = parent[v] < 0 ? (T)0 : (T)(1.0 / pw[v]);
    }
}
template <typename T>
__global__ void k_layout_pad(long long N, int *__restrict__ perm, uint8_t *__restrict__ flags,
                             int *__restrict__ ptop, T *__restrict__ rpw, int *__restrict__ lcc) {
    GSTRIDE(i, N) {
        perm[i] = -1;
        flags[i] = SEG_TOP | SEG_BOT;
        ptop[i] = -1;
        rpw[i] = (T)0;
        lcc[i] = 0;
    }
}
__global__ void k_lc_count(long long n, const int *__restrict__ tptr, const int *__restrict__ tcol,
                           const int *__restrict__ parent, const int *__restrict__ heavy, const int *__restrict__ lp,
                           int *__restrict__ lcc, uint8_t *__restrict__ flags, int *__restrict__ lcmax) {
    GSTRIDE(u, n) {
        int c = 0;
        for (int a = tptr[u]; a < tptr[u + 1]; a++) {
            int v = tcol[a];
            if (parent[v] == u && v != heavy[u]) c++;
        }
        lcc[lp[u]] = c;
        if (c > 0) flags[lp[u]] |= SEG_LC;
        if (c > 2) atomicMax(lcmax, c);
    }
}
__global__ void k_lc_fill(long long n, const int *__restrict__ tptr, const int *__restrict__ tcol,
                          const int *__restrict__ parent, const int *__restrict__ heavy, const int *__restrict__ lp,
                          const int *__restrict__ lc_ptr, int *__restrict__ lc_pos, int *__restrict__ lc_owner) {
    GSTRIDE(u, n) {
        int o = lc_ptr[lp[u]];
        for (int a = tptr[u]; a < tptr[u + 1]; a++) {
            int v = tcol[a];
            if (parent[v] == u && v != heavy[u]) {
                lc_owner[o] = lp[u];
                lc_pos[o++] = lp[v];
            }
        }
    }
}

// Tile dependencies of the dataflow sweeps: a light child c of u links the tile of
// u (which needs c's subtree current in the up-sweep) and the tile of c (which
// needs u's potential in the down-sweep).
__global__ void k_dep_keys(long long n, const int *__restrict__ parent, const int *__restrict__ head,
                           const int *__restrict__ lp, int TN, int ntile_bits, unsigned long long *__restrict__ kup,
                           unsigned long long *__restrict__ kdn, int *__restrict__ flag) {
    GSTRIDE(v, n) {
        int p = parent[v];
        bool light = p >= 0 && head[v] == v;
        flag[v] = light ? 1 : 0;
        if (light) {
            unsigned long long a = (unsigned long long)(lp[p] / TN), b = (unsigned long long)(lp[v] / TN);
            kup[v] = (a << ntile_bits) | b;
            kdn[v] = (b << ntile_bits) | a;
        }
    }
}
__global__ void k_dep_compact(long long n, const int *__restrict__ flag, const int *__restrict__ pos,
                              const unsigned long long *__restrict__ kin, unsigned long long *__restrict__ kout,
                              int *__restrict__ vout) {
    GSTRIDE(v, n) if (flag[v]) {
        kout[pos[v]] = kin[v];
        vout[pos[v]] = 0;
    }
}
// after sorting: keep the first of equal keys, count per owning tile
__global__ void k_dep_unique(long long c, const unsigned long long *__restrict__ key, int ntile_bits,
                             int *__restrict__ keep, int *__restrict__ cnt) {
    GSTRIDE(i, c) {
        bool first = i == 0 || key[i] != key[i - 1];
        keep[i] = first ? 1 : 0;
        if (first) atomicAdd(&cnt[(int)(key[i] >> ntile_bits)], 1);
    }
}
__global__ void k_dep_fill(long long c, const unsigned long long *__restrict__ key, const int *__restrict__ keep,
                           const int *__restrict__ kpos, int ntile_bits, int *__restrict__ dep) {
    GSTRIDE(i, c) if (keep[i]) dep[kpos[i]] = (int)(key[i] & ((1ull << ntile_bits) - 1));
}

// ------------------------------------------------------------ CSR of L_P
__global__ void k_p_count(long long n, const int *__restrict__ rowptr, const int *__restrict__ ceid,
                          const uint8_t *__restrict__ mask, int *__restrict__ cnt) {
    GSTRIDE(v, n) {
        int c = 0;
        for (int p = rowptr[v]; p < rowptr[v + 1]; p++) c += mask[ceid[p]] != 0;
        cnt[v] = c;
    }
}
template <typename T>
__global__ void k_p_fill(long long n, const int *__restrict__ rowptr, const int *__restrict__ col,
                         const int *__restrict__ ceid, const double *__restrict__ w, const uint8_t *__restrict__ mask,
                         const int *__restrict__ prow, int *__restrict__ pcol, T *__restrict__ pval,
                         double *__restrict__ pval64, double *__restrict__ degP) {
    GSTRIDE(v, n) {
        int o = prow[v];
        double s = 0.0;
        for (int p = rowptr[v]; p < rowptr[v + 1]; p++) {
            int e = ceid[p];
            if (mask[e] != 0) {
                double x = w[e];
                pcol[o] = col[p];
                pval[o] = (T)x;
                pval64[o] = x;
                s += x;
                o++;
            }
        }
        degP[v] = s;
    }
}
__global__ void k_count_mask(long long m, const uint8_t *__restrict__ mask, int *__restrict__ cnt) {
    int c1 = 0, c2 = 0, c3 = 0;
    GSTRIDE(e, m) {
        uint8_t x = mask[e];
        c1 += x == 1;
        c2 += x == 2;
        c3 += x > 2;
    }
    if (c1) atomicAdd(&cnt[0], c1);
    if (c2) atomicAdd(&cnt[1], c2);
    if (c3) atomicAdd(&cnt[2], c3);
}

}  // namespace


// ======================================================================= host

void plan_topo(Arena &a, const Dims &d, Topo &t, SetupTmp &st) {
    long long n = d.n, m = d.m;
    long long m2 = std::max<long long>(2 * m, 2 * n + 2);
    t.n = n;
    t.m = m;
    t.rowptr = a.take<int>(n + 1);
    t.col = a.take<int>(2 * m);
    t.ceid = a.take<int>(2 * m);
    t.degG = a.take<double>(n);
    t.devflags = a.take<unsigned>(4);
    t.scal_i = a.take<int>(32);
    t.mask = a.take<uint8_t>(m);
    t.prow = a.take<int>(n + 1);
    t.pcol = a.take<int>(2 * m);
    t.pval64 = a.take<double>(2 * m);
    t.degP = a.take<double>(n);
    t.parent = a.take<int>(n);
    t.heavy = a.take<int>(n);
    t.head = a.take<int>(n);
    t.off = a.take<int>(n);
    t.ld = a.take<int>(n);
    t.lp = a.take<int>(n);
    t.pw = a.take<double>(n);
    t.perm = a.take<int>(d.Npad + 1);
    t.flags = a.take<uint8_t>(d.Npad + 1);
    t.ptop = a.take<int>(d.Npad + 1);
    t.lc_ptr = a.take<int>(d.Npad + 1);
    t.lc_pos = a.take<int>(n);
    t.lc_owner = a.take<int>(n);
    t.lcmax = a.take<int>(1);
    t.done = a.take<unsigned>(d.ntiles);
    t.tickets = a.take<int>(2 * kMaxLevels);
    t.epoch_dev = a.take<unsigned>(4);
    t.lvl_tile = a.take<int>(kMaxLevels + 1);
    t.dep_up_ptr = a.take<int>(d.ntiles + 1);
    t.dep_dn_ptr = a.take<int>(d.ntiles + 1);
    t.dep_up = a.take<int>(n);
    t.dep_dn = a.take<int>(n);
    plan_scan(a, std::max<long long>(m2, d.Npad + 1) + 1, t.scan);
    plan_sort(a, std::max(m, n), t.sort);
    t.greedy_mark = a.take<int>(n);
    t.greedy_owner = a.take<int>(n);
    t.cand_acc = a.take<uint8_t>(m);
    t.keys = a.take<unsigned long long>(std::max(m, n));
    t.tmpA = a.take<int>(m2);  // candidate list / selection scratch
    t.tmpB = a.take<int>(m2);
    for (int i = 0; i < 12; i++) st.n1[i] = a.take<int>(n + 1);
    for (int i = 0; i < 10; i++) st.a1[i] = a.take<int>(m2);
    st.ku = a.take<unsigned long long>(std::max(m, n));
    st.lvl = a.take<long long>(2 * (kMaxLevels + 1));
}

int read_i32(const int *p, hipStream_t s) {
    int v = 0;
    GR_HIP(hipMemcpyAsync(&v, p, sizeof(int), hipMemcpyDeviceToHost, s));
    GR_HIP(hipStreamSynchronize(s));
    return v;
}

void validate_graph(Topo &t, hipStream_t s) {
    require(t.n >= 2 && t.m >= 1, GRASS_ERR_INVALID, "graph needs n >= 2 and m >= 1");
    require(t.n < (1ll << 30) && t.m < (1ll << 29), GRASS_ERR_INVALID, "graph too large for the int32 layout");
    fill_u32(t.devflags, 4, 0u, s);
    hipLaunchKernelGGL(k_validate, dim3(grid_for(t.m)), dim3(256), 0, s, t.n, t.m, t.src, t.dst, t.w, t.devflags);
    GR_CHECK_LAUNCH();
    unsigned f = (unsigned)read_i32((const int *)t.devflags, s);
    require(!(f & VF_RANGE), GRASS_ERR_INVALID, "edge ids out of range or src >= dst");
    require(!(f & VF_ORDER), GRASS_ERR_INVALID, "edges not sorted by (src, dst) or duplicated");
    require(!(f & VF_WEIGHT), GRASS_ERR_INVALID, "edge weights must be finite and > 0");
}

template <typename T>
__global__ void k_ell_fill(long long n, int E, const int *__restrict__ rowptr, const int *__restrict__ col,
                           const T *__restrict__ val, int *__restrict__ ecol, T *__restrict__ eval,
                           int *__restrict__ edeg, int *__restrict__ lcount, int *__restrict__ lrow, int cap) {
    GSTRIDE(v, n) {
        const int p0 = rowptr[v], d = rowptr[v + 1] - p0;
        int dd = d;
        if (d > kLongRow) {  // list order is arbitrary; each row's sum does not depend on it
            const int li = atomicAdd(lcount, 1);
            if (li < cap) {
                lrow[li] = (int)v;
                dd = -(li + 1);
            }
        }
        edeg[v] = dd;
        for (int e = 0; e < E; e++) {
            const bool h = e < d;
            ecol[v * E + e] = h ? col[p0 + e] : (int)v;
            eval[v * E + e] = h ? val[p0 + e] : (T)0;
        }
    }
}
// rows longer than 4 and longer than 6 entries
__global__ void k_count_long(long long n, const int *__restrict__ rowptr, int *__restrict__ cnt) {
    int c4 = 0, c6 = 0;
    GSTRIDE(v, n) {
        const int d = rowptr[v + 1] - rowptr[v];
        c4 += d > 4;
        c6 += d > 6;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        c4 += __shfl_xor(c4, off, 64);
        c6 += __shfl_xor(c6, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (c4) atomicAdd(&cnt[0], c4);
        if (c6) atomicAdd(&cnt[1], c6);
    }
}

// Padded width of the rows of L_G: the narrowest of 4, 6, 8 entries that holds
// whole rows for all but 1% of them (the rest continue in the CSR). A product
// gathers E rows per row whatever its length, so padding costs bandwidth: the
// 100^3 mesh (at most 6 neighbours) takes 6, the grid with long-range edges 6.
int choose_ell_width(long long n, const int *rowptr, int *cnt, hipStream_t s) {
    fill_i32(cnt, 2, 0, s);
    hipLaunchKernelGGL(k_count_long, dim3(grid_for(n)), dim3(256), 0, s, n, rowptr, cnt);
    GR_CHECK_LAUNCH();
    int h[2] = {0, 0};
    GR_HIP(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    GR_HIP(hipStreamSynchronize(s));
    if (h[0] * 100ll <= n) return 4;
    if (h[1] * 100ll <= n) return 6;
    return 8;
}

template <typename T>
void fill_ell(long long n, const int *rowptr, const int *col, const T *val, Ell<T> &e, hipStream_t s) {
    fill_i32(e.lcount, 1, 0, s);
    hipLaunchKernelGGL(k_ell_fill<T>, dim3(grid_for(n)), dim3(256), 0, s, n, e.E, rowptr, col, val, e.col, e.val,
                       e.deg, e.lcount, e.lrow, e.cap);
    GR_CHECK_LAUNCH();
    e.nlong = read_i32(e.lcount, s);
    require(e.nlong <= e.cap, GRASS_ERR_DEVICE, "long-row list exceeds its bound");
}

template <typename T>
void build_csr(Topo &t, Vecs<T> &v, SetupTmp &st, hipStream_t s) {
    long long n = t.n, m = t.m;
    int *in_cnt = st.n1[0], *out_cnt = st.n1[1], *in_first = st.n1[2], *out_first = st.n1[3], *tot = st.n1[4];
    fill_i32(in_cnt, n + 1, 0, s);
    fill_i32(out_cnt, n + 1, 0, s);
    hipLaunchKernelGGL(k_count_deg, dim3(grid_for(m)), dim3(256), 0, s, m, t.src, t.dst, in_cnt, out_cnt);
    GR_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_add2, dim3(grid_for(n + 1)), dim3(256), 0, s, n + 1, in_cnt, out_cnt, tot);
    GR_CHECK_LAUNCH();
    scan_excl_i32(tot, t.rowptr, n + 1, nullptr, t.scan, s);
    scan_excl_i32(in_cnt, in_first, n + 1, nullptr, t.scan, s);
    scan_excl_i32(out_cnt, out_first, n + 1, nullptr, t.scan, s);
    // in-edges of every node in ascending source order: stable sort of edge ids by dst
    int *vals = st.a1[0];
    hipLaunchKernelGGL(k_keys_dst, dim3(grid_for(m)), dim3(256), 0, s, m, t.dst, st.ku, vals);
    GR_CHECK_LAUNCH();
    int bits = 1;
    while ((1ll << bits) < n) bits++;
    radix_sort_pairs(st.ku, vals, m, bits, t.sort, s);
    hipLaunchKernelGGL(k_csr_out, dim3(grid_for(m)), dim3(256), 0, s, m, t.src, t.dst, t.rowptr, in_cnt, out_first,
                       t.col, t.ceid);
    GR_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_csr_in, dim3(grid_for(m)), dim3(256), 0, s, m, vals, t.src, t.dst, t.rowptr, in_first,
                       t.col, t.ceid);
    GR_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_row_finish<T>, dim3(grid_for(n)), dim3(256), 0, s, n, t.rowptr, t.ceid, t.w, v.cval, t.degG);
    GR_CHECK_LAUNCH();
    v.eg.E = choose_ell_width(n, t.rowptr, v.eg.lcount, s);  // within the kEllG slots planned
    fill_ell<T>(n, t.rowptr, t.col, v.cval, v.eg, s);
    hipLaunchKernelGGL(k_cast_w<T>, dim3(grid_for(m)), dim3(256), 0, s, m, t.w, v.wT);
    GR_CHECK_LAUNCH();
}

void boruvka(Topo &t, SetupTmp &st, uint8_t *tree, hipStream_t s) {
    long long n = t.n, m = t.m;
    int *comp = st.n1[0], *nxt = st.n1[1], *nxt2 = st.n1[2], *fin = st.n1[3], *be = st.n1[4];
    unsigned long long *bw = st.ku;
    int *counter = t.scal_i;
    fill_u8(tree, m, 0, s);
    hipLaunchKernelGGL(k_bor_init, dim3(grid_for(n)), dim3(256), 0, s, n, comp);
    GR_CHECK_LAUNCH();
    for (int round = 0; round < 64; round++) {
        fill_i32(counter, 1, 0, s);
        hipLaunchKernelGGL(k_bor_reset, dim3(grid_for(n)), dim3(256), 0, s, n, bw, be);
        hipLaunchKernelGGL(k_bor_maxw, dim3(grid_for(m)), dim3(256), 0, s, m, t.src, t.dst, t.w, comp, bw);
        hipLaunchKernelGGL(k_bor_mine, dim3(grid_for(m)), dim3(256), 0, s, m, t.src, t.dst, t.w, comp, bw, be);
        hipLaunchKernelGGL(k_bor_hook, dim3(grid_for(n)), dim3(256), 0, s, n, t.src, t.dst, comp, be, nxt, tree,
                           counter);
        hipLaunchKernelGGL(k_bor_break, dim3(grid_for(n)), dim3(256), 0, s, n, comp, nxt, nxt2);
        hipLaunchKernelGGL(k_bor_find, dim3(grid_for(n)), dim3(256), 0, s, n, comp, nxt2, fin, t.devflags);
        hipLaunchKernelGGL(k_bor_relabel, dim3(grid_for(n)), dim3(256), 0, s, n, comp, fin);
        GR_CHECK_LAUNCH();
        if (read_i32(counter, s) == 0) break;
    }
    unsigned f = (unsigned)read_i32(reinterpret_cast<const int *>(t.devflags), s);
    require(!(f & DEVERR_TREE), GRASS_ERR_DEVICE, "Boruvka hook forest has a cycle");
    long long cnt[3];
    count_mask(t, tree, cnt, s);
    require(cnt[0] == n - 1, GRASS_ERR_DISCONNECTED,
            "graph is not connected (" + std::to_string(n - cnt[0]) + " components)");
}

template <typename T>
void build_tree(Topo &t, Vecs<T> &v, const Dims &d, SetupTmp &st, hipStream_t s) {
    long long n = t.n, L = 2 * (n - 1);
    const int root = 0;
    int *counter = t.scal_i;
    int *total = t.scal_i + 8;
    // n-arrays
    int *tptr = st.n1[0], *tcnt = st.n1[1], *fpos = st.n1[2], *bpos = st.n1[3], *size = st.n1[4];
    int *anc2 = st.n1[5], *dist2 = st.n1[6], *plen = st.n1[7], *is_head = st.n1[8], *hpos = st.n1[9];
    int *pbase = st.n1[10], *lvl_nodes = st.n1[11];
    // arc arrays
    int *tcol = st.a1[0], *teid = st.a1[1], *tsrc = st.a1[2], *twin = st.a1[3];
    int *nxA = st.a1[4], *nxB = st.a1[5], *rkA = st.a1[6], *rkB = st.a1[7], *tval = st.a1[8], *tscan = st.a1[9];
    // tree adjacency (rows sorted by neighbour, inherited from the CSR of G)
    hipLaunchKernelGGL(k_tree_count, dim3(grid_for(n)), dim3(256), 0, s, n, t.rowptr, t.ceid, t.mask, tcnt);
    GR_CHECK_LAUNCH();
    fill_i32(tcnt + n, 1, 0, s);
    scan_excl_i32(tcnt, tptr, n + 1, total, t.scan, s);
    int arcs = read_i32(total, s);
    require(arcs == L, GRASS_ERR_INVALID, "tree edges (mask value 1) must number n-1 and span the graph");
    hipLaunchKernelGGL(k_tree_fill, dim3(grid_for(n)), dim3(256), 0, s, n, t.rowptr, t.col, t.ceid, t.mask, tptr,
                       tcol, teid, tsrc);
    hipLaunchKernelGGL(k_euler_succ, dim3(grid_for(L)), dim3(256), 0, s, L, tptr, tcol, tsrc, twin, nxA);
    hipLaunchKernelGGL(k_euler_cut, dim3(1), dim3(1), 0, s, tptr, twin, nxA, root);
    GR_CHECK_LAUNCH();
    // list ranking: rk = arcs after a in the tour
    hipLaunchKernelGGL(k_rank_init, dim3(grid_for(L)), dim3(256), 0, s, L, nxA, nxB, rkA);
    GR_CHECK_LAUNCH();
    int *cnx = nxB, *crk = rkA, *onx = nxA, *ork = rkB;
    int rounds = 1;
    while ((1ll << rounds) < L) rounds++;
    for (int r = 0; r <= rounds; r++) {
        hipLaunchKernelGGL(k_rank_jump, dim3(grid_for(L)), dim3(256), 0, s, L, cnx, crk, onx, ork);
        GR_CHECK_LAUNCH();
        std::swap(cnx, onx);
        std::swap(crk, ork);
    }
    int *rk = crk;
    // orientation
    fill_i32(t.parent, n, -1, s);
    fill_f64(t.pw, n, 0.0, s);
    fill_i32(counter, 1, 0, s);
    hipLaunchKernelGGL(k_orient, dim3(grid_for(L)), dim3(256), 0, s, L, tsrc, tcol, teid, twin, rk, t.w, t.parent,
                       t.pw, fpos, bpos, counter);
    GR_CHECK_LAUNCH();
    int oriented = read_i32(counter, s);
    require(oriented == n - 1, GRASS_ERR_INVALID, "tree edges (mask value 1) do not form a spanning tree");
    hipLaunchKernelGGL(k_sizes, dim3(grid_for(n)), dim3(256), 0, s, n, fpos, bpos, t.parent, size);
    hipLaunchKernelGGL(k_heavy, dim3(grid_for(n)), dim3(256), 0, s, n, tptr, tcol, t.parent, size, t.heavy);
    GR_CHECK_LAUNCH();
    // heads and offsets along heavy paths by pointer doubling
    hipLaunchKernelGGL(k_hl_init, dim3(grid_for(n)), dim3(256), 0, s, n, t.parent, t.heavy, t.head, t.off);
    GR_CHECK_LAUNCH();
    int *changed = t.scal_i + 4;
    int *ca = t.head, *cd = t.off, *oa = anc2, *od = dist2;
    for (int r = 0; r < 40; r++) {
        fill_i32(changed, 1, 0, s);
        hipLaunchKernelGGL(k_hl_jump, dim3(grid_for(n)), dim3(256), 0, s, n, ca, cd, oa, od, changed);
        GR_CHECK_LAUNCH();
        std::swap(ca, oa);
        std::swap(cd, od);
        if (read_i32(changed, s) == 0) break;
    }
    if (ca != t.head) {
        GR_HIP(hipMemcpyAsync(t.head, ca, n * sizeof(int), hipMemcpyDeviceToDevice, s));
        GR_HIP(hipMemcpyAsync(t.off, cd, n * sizeof(int), hipMemcpyDeviceToDevice, s));
    }
    // light depth from a prefix sum over the Euler tour
    hipLaunchKernelGGL(k_tour_vals, dim3(grid_for(L)), dim3(256), 0, s, L, tsrc, tcol, twin, rk, t.parent, t.head,
                       tval);
    GR_CHECK_LAUNCH();
    scan_incl_i32(tval, tscan, L, t.scan, s);
    hipLaunchKernelGGL(k_light_depth, dim3(grid_for(n)), dim3(256), 0, s, n, t.parent, fpos, tscan, t.ld);
    GR_CHECK_LAUNCH();
    // path lengths and level sizes
    fill_i32(plen, n, 0, s);
    hipLaunchKernelGGL(k_path_len, dim3(grid_for(n)), dim3(256), 0, s, n, t.head, t.off, plen);
    fill_i32(lvl_nodes, kMaxLevels + 2, 0, s);
    int *maxld = lvl_nodes + kMaxLevels;
    hipLaunchKernelGGL(k_level_stats, dim3(grid_for(n)), dim3(256), 0, s, n, t.head, t.ld, plen, lvl_nodes, maxld,
                       is_head);
    GR_CHECK_LAUNCH();
    std::vector<int> hl(kMaxLevels + 2);
    GR_HIP(hipMemcpyAsync(hl.data(), lvl_nodes, (kMaxLevels + 2) * sizeof(int), hipMemcpyDeviceToHost, s));
    GR_HIP(hipStreamSynchronize(s));
    int nlev = hl[kMaxLevels] + 1;
    require(nlev >= 1 && nlev <= kMaxLevels, GRASS_ERR_DEVICE, "tree light depth exceeds the layout limit");
    t.nlev = nlev;
    t.lvl_start.assign(nlev + 1, 0);
    std::vector<long long> both(2 * (nlev + 1), 0);
    for (int l = 0; l < nlev; l++) {
        long long len = hl[l];
        long long padded = (len + d.TN - 1) / d.TN * d.TN;
        t.lvl_start[l + 1] = t.lvl_start[l] + padded;
        both[nlev + 1 + l + 1] = both[nlev + 1 + l] + len;
    }
    for (int l = 0; l <= nlev; l++) both[l] = t.lvl_start[l];
    t.N = t.lvl_start[nlev];
    require(t.N <= d.Npad, GRASS_ERR_DEVICE, "layout exceeds its bound");
    // path heads sorted by (light depth, node id)
    scan_excl_i32(is_head, hpos, n, total, t.scan, s);
    int nh = read_i32(total, s);
    int *heads = tscan;  // tour scan consumed by k_light_depth
    hipLaunchKernelGGL(k_head_keys, dim3(grid_for(n)), dim3(256), 0, s, n, is_head, hpos, t.ld, st.ku, heads);
    GR_CHECK_LAUNCH();
    radix_sort_pairs(st.ku, heads, nh, 8, t.sort, s);
    int *hlen = tval;
    hipLaunchKernelGGL(k_gather_plen, dim3(grid_for(nh)), dim3(256), 0, s, (long long)nh, heads, plen, hlen);
    GR_CHECK_LAUNCH();
    int *cum = hpos;
    scan_excl_i32(hlen, cum, nh, nullptr, t.scan, s);
    GR_HIP(hipMemcpyAsync(st.lvl, both.data(), both.size() * sizeof(long long), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_path_base, dim3(grid_for(nh)), dim3(256), 0, s, (long long)nh, heads, cum, t.ld, st.lvl,
                       st.lvl + nlev + 1, pbase);
    GR_CHECK_LAUNCH();
    // layout arrays
    hipLaunchKernelGGL(k_layout_pad<T>, dim3(grid_for(t.N + 1)), dim3(256), 0, s, t.N + 1, t.perm, t.flags, t.ptop,
                       v.rpw, t.lc_ptr);
    hipLaunchKernelGGL(k_layout<T>, dim3(grid_for(n)), dim3(256), 0, s, n, t.head, t.off, pbase, t.heavy, t.parent,
                       t.pw, t.lp, t.perm, t.flags, t.ptop, v.rpw);
    fill_i32(t.lcmax, 1, 0, s);
    hipLaunchKernelGGL(k_lc_count, dim3(grid_for(n)), dim3(256), 0, s, n, tptr, tcol, t.parent, t.heavy, t.lp,
                       t.lc_ptr, t.flags, t.lcmax);
    GR_CHECK_LAUNCH();
    t.max_lc = read_i32(t.lcmax, s);
    scan_excl_i32(t.lc_ptr, t.lc_ptr, t.N + 1, nullptr, t.scan, s);
    hipLaunchKernelGGL(k_lc_fill, dim3(grid_for(n)), dim3(256), 0, s, n, tptr, tcol, t.parent, t.heavy, t.lp, t.lc_ptr,
                       t.lc_pos, t.lc_owner);
    GR_CHECK_LAUNCH();
    // per-level tile ranges and per-tile dependencies of the dataflow sweeps
    long long NT = t.N / d.TN;
    t.ntiles_used = NT;
    std::vector<int> lt(kMaxLevels + 1, 0);  // lives until the stream synchronizes below
    {
        for (int l = 0; l <= nlev; l++) lt[l] = (int)(t.lvl_start[l] / d.TN);
        GR_HIP(hipMemcpyAsync(t.lvl_tile, lt.data(), (nlev + 1) * sizeof(int), hipMemcpyHostToDevice, s));
        int bits = 1;
        while ((1ll << bits) < NT + 1) bits++;
        unsigned long long *kup = reinterpret_cast<unsigned long long *>(st.a1[0]);  // tcol no longer needed
        unsigned long long *kdn = reinterpret_cast<unsigned long long *>(st.a1[2]);  // tsrc no longer needed
        int *flag = st.n1[0], *fpos2 = st.n1[1];
        hipLaunchKernelGGL(k_dep_keys, dim3(grid_for(n)), dim3(256), 0, s, n, t.parent, t.head, t.lp, d.TN, bits, kup,
                           kdn, flag);
        GR_CHECK_LAUNCH();
        fill_i32(flag + n, 1, 0, s);
        scan_excl_i32(flag, fpos2, n + 1, total, t.scan, s);
        int c = read_i32(total, s);
        for (int dir = 0; dir < 2; dir++) {
            unsigned long long *kin = dir == 0 ? kup : kdn;
            int *ptr = dir == 0 ? t.dep_up_ptr : t.dep_dn_ptr;
            int *dep = dir == 0 ? t.dep_up : t.dep_dn;
            int *cntv = st.n1[2], *keep = st.a1[4], *kpos = st.a1[5];
            fill_i32(cntv, NT + 1, 0, s);
            if (c > 0) {
                hipLaunchKernelGGL(k_dep_compact, dim3(grid_for(n)), dim3(256), 0, s, n, flag, fpos2, kin, st.ku,
                                   st.a1[6]);
                GR_CHECK_LAUNCH();
                radix_sort_pairs(st.ku, st.a1[6], c, 2 * bits, t.sort, s);
                hipLaunchKernelGGL(k_dep_unique, dim3(grid_for(c)), dim3(256), 0, s, (long long)c, st.ku, bits, keep,
                                   cntv);
                GR_CHECK_LAUNCH();
                scan_excl_i32(keep, kpos, c, nullptr, t.scan, s);
                hipLaunchKernelGGL(k_dep_fill, dim3(grid_for(c)), dim3(256), 0, s, (long long)c, st.ku, keep, kpos,
                                   bits, dep);
                GR_CHECK_LAUNCH();
            }
            scan_excl_i32(cntv, ptr, NT + 1, nullptr, t.scan, s);
        }
    }
    fill_u32(t.done, d.ntiles, 0u, s);
    fill_u32(reinterpret_cast<unsigned *>(v.aggw), 2 * d.ntiles * d.kp * (long long)(sizeof(T) / 4), 0u, s);
    fill_u32(t.epoch_dev, 4, 0u, s);
    t.epoch = 0;
    GR_HIP(hipStreamSynchronize(s));
}

template <typename T>
void build_pcsr(Topo &t, Vecs<T> &v, hipStream_t s) {
    long long n = t.n;
    int *cnt = t.tmpB;
    hipLaunchKernelGGL(k_p_count, dim3(grid_for(n)), dim3(256), 0, s, n, t.rowptr, t.ceid, t.mask, cnt);
    GR_CHECK_LAUNCH();
    fill_i32(cnt + n, 1, 0, s);
    scan_excl_i32(cnt, t.prow, n + 1, nullptr, t.scan, s);
    hipLaunchKernelGGL(k_p_fill<T>, dim3(grid_for(n)), dim3(256), 0, s, n, t.rowptr, t.col, t.ceid, t.w, t.mask,
                       t.prow, t.pcol, v.pval, t.pval64, t.degP);
    GR_CHECK_LAUNCH();
    fill_ell<T>(n, t.prow, t.pcol, v.pval, v.ep, s);
}

void count_mask(Topo &t, const uint8_t *mask, long long out[3], hipStream_t s) {
    fill_i32(t.scal_i + 12, 3, 0, s);
    hipLaunchKernelGGL(k_count_mask, dim3(grid_for(t.m)), dim3(256), 0, s, t.m, mask, t.scal_i + 12);
    GR_CHECK_LAUNCH();
    int h[3];
    GR_HIP(hipMemcpyAsync(h, t.scal_i + 12, sizeof(h), hipMemcpyDeviceToHost, s));
    GR_HIP(hipStreamSynchronize(s));
    out[0] = h[0];
    out[1] = h[1];
    out[2] = h[2];
}

template void build_csr<float>(Topo &, Vecs<float> &, SetupTmp &, hipStream_t);
template void build_csr<double>(Topo &, Vecs<double> &, SetupTmp &, hipStream_t);
template void build_tree<float>(Topo &, Vecs<float> &, const Dims &, SetupTmp &, hipStream_t);
template void build_tree<double>(Topo &, Vecs<double> &, const Dims &, SetupTmp &, hipStream_t);
template void build_pcsr<float>(Topo &, Vecs<float> &, hipStream_t);
template void build_pcsr<double>(Topo &, Vecs<double> &, hipStream_t);

}  // namespace grass
