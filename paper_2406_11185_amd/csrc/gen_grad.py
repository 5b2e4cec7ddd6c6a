"""Generate the per-class nuclear-gradient code (derivative integrals) for the HIP kernels.

The derivative of a contracted Cartesian Gaussian with respect to its centre,
  d/dA_i [x_A^l e^{-a r_A^2}] = 2a x_A^{l+1} e^{-a r_A^2} - l_i x_A^{l-1} e^{-a r_A^2},
turns each derivative integral into integrals with one angular momentum more
(weighted by twice the primitive exponent) minus integrals with one less.  Per
shell quartet the kernel accumulates, over all primitive quartets, the
contracted vertical-recurrence integrals [e0|f0] of total order L+1 in four
sets:
  GA  weight 2a   e in levels [la+1, la+lb+1], f in [lc, lc+ld]
  GB  weight 2b   e in levels [la, la+lb+1],   f in [lc, lc+ld]
  GC  weight 2c   e in levels [la, la+lb],     f in [lc+1, lc+ld+1]
  GU  weight 1    e in levels [la-1, la+lb],   f in [lc-1, lc+ld]
The horizontal recurrences then give (a+1_i b|cd), (a b+1_i|cd), (ab|c+1_i d) and
the lower-order (a-1_i b|cd), (a b-1_i|cd), (ab|c-1_i d), which are contracted
with Gamma_abcd = 1/2 D_ab D_cd - 1/8 (D_ac D_bd + D_ad D_bc).  The derivative
with respect to the fourth centre follows from translational invariance.

The accumulators are built in balanced passes of at most PASS_ACC values (one
pass of the primitive loop each) and parked in a global workspace, as in the
multi-pass energy classes.
"""
from __future__ import annotations

import json
import os
import sys

import gen_hgp as g

# (measured on gfx950 for the 270-function molecule: passes of <= 96 weighted
# accumulators 191 ms per gradient, <= 64 215 ms, <= 128 203 ms)
PASS_ACC = 96
XYZ = "xyz"


def levels(lo, hi):
    lo = max(lo, 0)
    return [c for l in range(lo, hi + 1) for c in g.cart(l)] if hi >= lo else []


def cart_index(l):
    return {c: i for i, c in enumerate(g.cart(l))}


class BraH(g.Code):
    """(a b| of shell pair (la, lb) from the vector (e 0| with e in levels [la, la+lb])."""

    def __init__(self, la, lb):
        super().__init__("b")
        self.E = {c: i for i, c in enumerate(levels(la, la + lb))}

    def node(self, a, b):
        key = (a, b)
        if key in self.memo:
            return self.memo[key]
        if sum(b) > 0:
            i = next(k for k in range(3) if b[k] > 0)
            x = self.node(g.add(a, i), g.sub(b, i))
            y = self.node(a, g.sub(b, i))
            name = self.emit(f"{x} + AB{XYZ[i]} * {y}", 2)
        else:
            name = f"e[{self.E[a]}]"
        self.memo[key] = name
        return name


class KetH(g.Code):
    def __init__(self, lc, ld):
        super().__init__("k")
        self.F = {c: i for i, c in enumerate(levels(lc, lc + ld))}

    def node(self, c, d):
        key = (c, d)
        if key in self.memo:
            return self.memo[key]
        if sum(d) > 0:
            i = next(k for k in range(3) if d[k] > 0)
            x = self.node(g.add(c, i), g.sub(d, i))
            y = self.node(c, g.sub(d, i))
            name = self.emit(f"{x} + CD{XYZ[i]} * {y}", 2)
        else:
            name = f"f[{self.F[c]}]"
        self.memo[key] = name
        return name


def bra_fn(name, la, lb):
    h = BraH(la, lb)
    outs = []
    for ia, a in enumerate(g.cart(la)):
        for ib, b in enumerate(g.cart(lb)):
            outs.append(f"out[{ia * g.ncart(lb) + ib}] = {h.node(a, b)};")
    s = ["  template <typename T>",
         f"  __device__ __forceinline__ static void {name}(const T* __restrict__ e, T ABx, T ABy, T ABz,"
         " T* __restrict__ out) {",
         "    (void)ABx; (void)ABy; (void)ABz;"]
    s += ["    " + x for x in h.lines] + ["    " + x for x in outs] + ["  }"]
    return s, h.flops


def ket_fn(name, lc, ld):
    h = KetH(lc, ld)
    outs = []
    for ic, c in enumerate(g.cart(lc)):
        for id_, d in enumerate(g.cart(ld)):
            outs.append(f"out[{ic * g.ncart(ld) + id_}] = {h.node(c, d)};")
    s = ["  template <typename T>",
         f"  __device__ __forceinline__ static void {name}(const T* __restrict__ f, T CDx, T CDy, T CDz,"
         " T* __restrict__ out) {",
         "    (void)CDx; (void)CDy; (void)CDz;"]
    s += ["    " + x for x in h.lines] + ["    " + x for x in outs] + ["  }"]
    return s, h.flops


def grad_lanes(ng, npass):
    """Lanes that share one shell quartet: 1 for the lightest classes, 4 for up to
    four passes, 16 beyond."""
    if ng <= 32:
        return 1
    return 4 if npass <= 4 else 16


def gen_grad_class(la, lb, lc, ld):
    name = g.cls_name(la, lb, lc, ld)
    L1 = la + lb + lc + ld + 1
    na, nb, nc, nd = g.ncart(la), g.ncart(lb), g.ncart(lc), g.ncart(ld)
    use_u = (la + lb + lc) > 0
    sets = [("A", "wA", levels(la + 1, la + lb + 1), levels(lc, lc + ld)),
            ("B", "wB", levels(la, la + lb + 1), levels(lc, lc + ld)),
            ("C", "wC", levels(la, la + lb), levels(lc + 1, lc + ld + 1))]
    if use_u:
        sets.append(("U", None, levels(la - 1, la + lb), levels(lc - 1, lc + ld)))
    off = {}
    o = 0
    for nm, w, Es, Fs in sets:
        off[nm] = o
        o += len(Es) * len(Fs)
    NG = o
    # unique VRR nodes with their consumers, ordered by e then f: a pass then
    # holds a few bra components with all their ket components, which shares
    # more of the recurrence tree within the pass than blocks of ket components
    # do (about half the recurrence work summed over the passes for (dd|dp))
    nodes = {}
    for nm, w, Es, Fs in sets:
        for ie, e in enumerate(Es):
            for jf, f in enumerate(Fs):
                nodes.setdefault((f, e), []).append((w, off[nm] + ie * len(Fs) + jf))
    order = sorted(nodes, key=lambda fe: (sum(fe[1]), fe[1], sum(fe[0]), fe[0]))
    # balanced passes of at most PASS_ACC accumulators
    total = sum(len(v) for v in nodes.values())
    cap = -(-total // -(-total // PASS_ACC))
    passes, cur, cnt = [], [], 0
    for fe in order:
        k = len(nodes[fe])
        if cnt + k > cap and cur:
            passes.append(cur)
            cur, cnt = [], 0
        cur.append(fe)
        cnt += k
    if cur:
        passes.append(cur)

    s = [f"// gradient class ({g.LNAME[la]}{g.LNAME[lb]}|{g.LNAME[lc]}{g.LNAME[ld]}): "
         f"{NG} weighted accumulators in {len(passes)} passes",
         f"struct GCls_{name} {{",
         f"  static constexpr int LA = {la}, LB = {lb}, LC = {lc}, LD = {ld}, L = {L1};",
         f"  static constexpr int NA = {na}, NB = {nb}, NC = {nc}, ND = {nd}, NG = {NG};",
         f"  static constexpr int NPASS = {len(passes)}, USE_U = {1 if use_u else 0};",
         f"  static constexpr int GMAX = {grad_lanes(NG, len(passes))};  // most lanes per shell quartet"]
    # set geometry
    for nm, w, Es, Fs in sets:
        s.append(f"  static constexpr int OFF_{nm} = {off[nm]}, NE_{nm} = {len(Es)}, NF_{nm} = {len(Fs)};")
    if not use_u:
        s.append("  static constexpr int OFF_U = 0, NE_U = 0, NF_U = 0;")
    vrr_flops = 0
    one = g.VRR(L1)
    for fe in order:
        one.node(fe[1], fe[0], 0)
    vrr_flops_alg = one.flops + sum(len(v) for v in nodes.values()) * 2
    for j, pas in enumerate(passes):
        v = g.VRR(L1)
        lines, store = [], []
        k = 0
        for fe in pas:
            val = v.node(fe[1], fe[0], 0)
            for w, gi in nodes[fe]:
                # accumulate right after the value is formed: few live temporaries
                v.lines.append(f"acc[{k}] += {w} * {val};" if w else f"acc[{k}] += {val};")
                store.append(f"G[z + {gi}] = acc[{k}];")
                k += 1
        vrr_flops += v.flops + 2 * k
        s.append(f"  static constexpr int PASS{j}_N = {k};")
        s.append("  template <typename T>")
        s.append(f"  __device__ __forceinline__ static void vrr_p{j}(const T* __restrict__ F, const VrrCoef<T>& c,"
                 " T wA, T wB, T wC, T* __restrict__ acc) {")
        s += ["    " + x for x in g.VRR_PROLOGUE]
        s.append("    (void)wA; (void)wB; (void)wC;")
        s += ["    " + x for x in v.lines] + ["    " + x for x in lines] + ["  }"]
        s.append("  template <typename T, class A>")
        s.append(f"  __device__ __forceinline__ static void store_p{j}(const T* __restrict__ acc, A G, int z) {{")
        s += ["    " + x for x in store] + ["  }"]
    s.append("  template <int J> struct Pass;")
    s.append("  template <int J, typename T>")
    s.append("  __device__ __forceinline__ static void vrr_pass(const T* __restrict__ F, const VrrCoef<T>& c,"
             " T wA, T wB, T wC, T* __restrict__ acc) {")
    for j in range(len(passes)):
        kw = "if" if j == 0 else "else if"
        s.append(f"    {kw} constexpr (J == {j}) vrr_p{j}<T>(F, c, wA, wB, wC, acc);")
    s.append("  }")
    s.append("  template <int J, typename T, class A>")
    s.append("  __device__ __forceinline__ static void store_pass(const T* __restrict__ acc, A G, int z) {")
    for j in range(len(passes)):
        kw = "if" if j == 0 else "else if"
        s.append(f"    {kw} constexpr (J == {j}) store_p{j}<T, A>(acc, G, z);")
    s.append("  }")
    # ket HRR shapes
    hrr_flops = 0
    k0, f0 = ket_fn("ket_b", lc, ld)
    s += k0
    hrr_flops += f0 * (len(sets[0][2]) + len(sets[1][2]) + (len(sets[3][2]) if use_u else 0))
    k1, f1 = ket_fn("ket_p", lc + 1, ld)
    s += k1
    hrr_flops += f1 * len(sets[2][2])
    s.append(f"  static constexpr int NCP = {g.ncart(lc + 1) * nd};")
    if lc >= 1:
        k2, f2 = ket_fn("ket_m", lc - 1, ld)
        s += k2
        hrr_flops += f2 * len(sets[3][2])
        s.append(f"  static constexpr int NCM = {g.ncart(lc - 1) * nd};")
    else:
        s.append("  static constexpr int NCM = 0;")
    # offsets of the sub-ranges inside U
    s.append(f"  static constexpr int U_FB = {g.ncart(lc - 1) if (use_u and lc >= 1) else 0};"
             "  // f of levels [lc, lc+ld] inside U's f list")
    s.append(f"  static constexpr int U_EB = {g.ncart(la - 1) if (use_u and la >= 1) else 0};"
             "  // e of levels [la, ...] inside U's e list")
    s.append(f"  static constexpr int NE_AM = {len(levels(la - 1, la + lb - 1)) if la >= 1 else 0};")
    s.append(f"  static constexpr int NE_BM = {len(levels(la, la + lb - 1)) if lb >= 1 else 0};")
    s.append(f"  static constexpr int NE_0 = {len(levels(la, la + lb))};")
    # bra HRR shapes
    fl_cd = 0
    b_ap, x = bra_fn("bra_ap", la + 1, lb); s += b_ap; fl_cd += x
    b_bp, x = bra_fn("bra_bp", la, lb + 1); s += b_bp; fl_cd += x
    b_0, x = bra_fn("bra_0", la, lb); s += b_0; fl_cd += 6 * x
    if la >= 1:
        b_am, x = bra_fn("bra_am", la - 1, lb); s += b_am; fl_cd += x
    if lb >= 1:
        b_bm, x = bra_fn("bra_bm", la, lb - 1); s += b_bm; fl_cd += x
    hrr_flops += fl_cd * nc * nd
    # component tables
    ca, cb, cc = g.cart(la), g.cart(lb), g.cart(lc)
    ia1, ib1, ic1 = cart_index(la + 1), cart_index(lb + 1), cart_index(lc + 1)
    iam = cart_index(la - 1) if la >= 1 else {}
    ibm = cart_index(lb - 1) if lb >= 1 else {}
    icm = cart_index(lc - 1) if lc >= 1 else {}
    s.append("  __device__ static constexpr int CPLUS[{}][3] = {{{}}};".format(
        nc, ", ".join("{" + ", ".join(str(ic1[g.add(c, i)]) for i in range(3)) + "}" for c in cc)))
    s.append("  __device__ static constexpr int CMINUS[{}][3] = {{{}}};".format(
        nc, ", ".join("{" + ", ".join(str(icm[g.sub(c, i)]) if c[i] > 0 else "0" for i in range(3)) + "}"
                      for c in cc)))
    s.append("  __device__ static constexpr int CPOW[{}][3] = {{{}}};".format(
        nc, ", ".join("{" + ", ".join(str(c[i]) for i in range(3)) + "}" for c in cc)))
    # contraction of one ket component pair (c, d): gA, gB from compile-time
    # bra components, gC from the runtime c via the tables
    body = []
    nb_ap, nb_bp = g.ncart(lb), g.ncart(lb + 1)
    for i in range(3):
        terms = []
        for ja, a in enumerate(ca):
            for jb, b in enumerate(cb):
                gam = f"Gam[{ja * nb + jb}]"
                terms.append(f"{gam} * double(xap[{ia1[g.add(a, i)] * nb_ap + jb}])")
                if la >= 1 and a[i] > 0:
                    terms.append(f"-{a[i]}.0 * {gam} * double(xam[{iam[g.sub(a, i)] * nb + jb}])")
        body.append(f"gA[{i}] += " + " + ".join(terms) + ";")
    for i in range(3):
        terms = []
        for ja, a in enumerate(ca):
            for jb, b in enumerate(cb):
                gam = f"Gam[{ja * nb + jb}]"
                terms.append(f"{gam} * double(xbp[{ja * nb_bp + ib1[g.add(b, i)]}])")
                if lb >= 1 and b[i] > 0:
                    terms.append(f"-{b[i]}.0 * {gam} * double(xbm[{ja * g.ncart(lb - 1) + ibm[g.sub(b, i)]}])")
        body.append(f"gB[{i}] += " + " + ".join(terms) + ";")
    s.append("  template <typename T>")
    s.append("  __device__ __forceinline__ static void contract_ab(const double* Gam, const T* xap,"
             " const T* xam, const T* xbp, const T* xbm, double* gA, double* gB) {")
    s.append("    (void)xam; (void)xbm;")
    s += ["    " + x for x in body] + ["  }"]
    s.append("  template <typename T>")
    s.append("  __device__ __forceinline__ static double dot0(const double* Gam, const T* x) {")
    s.append("    return " + " + ".join(f"Gam[{t}] * double(x[{t}])" for t in range(na * nb)) + ";")
    s.append("  }")
    dig = na * nb * nc * nd * (2 * 6 + 2 * 9 + 6)
    s.append(f"  static constexpr int VRR_FLOPS = {vrr_flops}, VRR_FLOPS_ALG = {vrr_flops_alg}, "
             f"HRR_FLOPS = {hrr_flops}, CONTRACT_FLOPS = {dig};")
    s.append("};")
    for j, pas in enumerate(passes):
        n = sum(len(nodes[fe]) for fe in pas)
        s.append(f"template <> struct GCls_{name}::Pass<{j}> {{ static constexpr int N = {n}; }};")
    ncd = nc * nd
    ws = (NG + len(sets[0][2]) * ncd + len(sets[1][2]) * ncd + len(sets[2][2]) * g.ncart(lc + 1) * nd
          + (len(sets[3][2]) * ncd + len(sets[3][2]) * (g.ncart(lc - 1) * nd if lc >= 1 else 0)
             if use_u else 0))
    s.insert(s.index("};"), f"  static constexpr int WS = {ws};  // workspace values per lane")
    info = dict(name=name, L=L1, ng=NG, npass=len(passes), vrr_flops=vrr_flops, ws=ws,
                lanes=grad_lanes(NG, len(passes)),
                vrr_flops_alg=vrr_flops_alg, hrr_flops=hrr_flops, contract_flops=dig)
    return "\n".join(s) + "\n", info


WS_WAVES = 4096                       # wavefronts the 1 GiB workspace should hold


def grad_lane_options(gmax, ws):
    """Lane counts a gradient class is compiled for; the host picks one per launch.
    Fewer lanes per quartet mean more quartets per wavefront and a larger FP64
    workspace: only counts whose workspace lets WS_WAVES wavefronts run."""
    return [x for x in (1, 4, 16) if x <= gmax and
            (x == gmax or (64 // x) * ws * 8 * WS_WAVES <= (1 << 30))]


def wrapper(name, gmax, ws):
    opts = grad_lane_options(gmax, ws)
    lines = ["// generated by gen_grad.py -- do not edit",
             '#include "jk_grad_device.hpp"',
             "namespace jk {",
             f'#include "gcls_{name}.inc"',
             f"void launch_grad_{name}(const GradLaunch& a, int fp32, hipStream_t s) {{",
             "  const dim3 grid((a.nwaves + kWavesPerBlock - 1) / kWavesPerBlock), block(kBlock);",
             "  const size_t lds = a.lds_bytes;"]
    for j, gl in enumerate(opts):
        cond = "true" if j == len(opts) - 1 else f"a.e.lanes == {gl}"
        lines += [f"  {'if' if j == 0 else 'else if'} ({cond}) {{",
                  f"    if (fp32) launch_kernel(&grad_kernel<GCls_{name}, float, {gl}>, grid, block, lds, s, a.e.dry != 0, a);",
                  f"    else launch_kernel(&grad_kernel<GCls_{name}, double, {gl}>, grid, block, lds, s, a.e.dry != 0, a);",
                  "  }"]
    lines += ["}", "}  // namespace jk", ""]
    return "\n".join(lines)


def table(names, infos):
    t = ["// generated by gen_grad.py -- do not edit", '#include "jk_grad_device.hpp"', "namespace jk {"]
    for n in names:
        t.append(f"void launch_grad_{n}(const GradLaunch&, int, hipStream_t);")
    t.append("int grad_ws_elems(int cls) {")
    t.append("  static const int w[21] = {" + ", ".join(str(i["ws"]) for i in infos) + "};")
    t.append("  return (cls >= 0 && cls < 21) ? w[cls] : 0;")
    t.append("}")
    t.append("// bit g set: the gradient class has a kernel with g lanes per shell quartet")
    t.append("int grad_lane_mask(int cls) {")
    t.append("  static const int m[21] = {" + ", ".join(
        str(sum(1 << x for x in grad_lane_options(i["lanes"], i["ws"]))) for i in infos) + "};")
    t.append("  return (cls >= 0 && cls < 21) ? m[cls] : 2;")
    t.append("}")
    t.append("int grad_lanes(int cls) {")
    t.append("  static const int g[21] = {" + ", ".join(str(i["lanes"]) for i in infos) + "};")
    t.append("  return (cls >= 0 && cls < 21) ? g[cls] : 1;")
    t.append("}")
    t.append("void launch_grad(int cls, int fp32, const GradLaunch& a, hipStream_t s) {")
    t.append("  switch (cls) {")
    for q, n in enumerate(names):
        t.append(f"    case {q}: launch_grad_{n}(a, fp32, s); break;")
    t += ["    default: break;", "  }", "}", "}  // namespace jk", ""]
    return "\n".join(t)


def main(outdir):
    os.makedirs(outdir, exist_ok=True)
    infos, names = [], []
    for X, Y, la, lb, lc, ld in g.quartet_classes():
        code, info = gen_grad_class(la, lb, lc, ld)
        infos.append(info)
        names.append(info["name"])
        g.write_if_changed(os.path.join(outdir, f"gcls_{info['name']}.inc"),
                           "// generated by gen_grad.py -- do not edit\n" + code)
        g.write_if_changed(os.path.join(outdir, f"gcls_{info['name']}.hip"), wrapper(info["name"], info["lanes"], info["ws"]))
    g.write_if_changed(os.path.join(outdir, "jk_grad_table.hip"), table(names, infos))
    g.write_if_changed(os.path.join(outdir, "grad_classes.json"), json.dumps(infos, indent=1))
    return infos


if __name__ == "__main__":
    for i in main(sys.argv[1] if len(sys.argv) > 1 else "generated"):
        print(i)
