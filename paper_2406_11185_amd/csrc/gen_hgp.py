"""Generate the per-class Head-Gordon-Pople integral code for the HIP kernels.

The paper's GPU design gives every angular-momentum combination its own
computational path produced by code generation ("Key Components Redesign and
Implementation", ERI paragraph, second item).  This script writes that code
as straight-line C++ for each of the 21 canonical shell-quartet classes over
s, p and Cartesian d shells:

  * vrr   -- Obara-Saika vertical recurrences (the HGP form) that build the
             primitive integrals [e0|f0]^(0) for |e| in [la, la+lb] and
             |f| in [lc, lc+ld] from the scaled Boys values (00|00)^(m) and add
             them to the contracted accumulators;
  * hrr   -- horizontal recurrences that move angular momentum from A to B
             and from C to D after contraction, fused with the J/K digestion;
  * diag  -- the same HRR restricted to the diagonal components (ab|ab), for
             the Cauchy-Schwarz bound of a shell pair.

Recurrences (P = Gaussian product centre of the bra, Q of the ket,
W = (pP + qQ)/(p+q), rho = pq/(p+q)):
  [e+1_i,0|f0]^m = PA_i [e0|f0]^m + WP_i [e0|f0]^{m+1}
                 + e_i/(2p) ([e-1_i,0|f0]^m - rho/p [e-1_i,0|f0]^{m+1})
                 + f_i/(2(p+q)) [e0|f-1_i,0]^{m+1}
  [e0|f+1_i,0]^m = QC_i [e0|f0]^m + WQ_i [e0|f0]^{m+1}
                 + f_i/(2q) ([e0|f-1_i,0]^m - rho/q [e0|f-1_i,0]^{m+1})
                 + e_i/(2(p+q)) [e-1_i,0|f0]^{m+1}
  (a, b+1_i| = (a+1_i, b| + AB_i (a, b|      |c, d+1_i) = |c+1_i, d) + CD_i |c, d)

It also reports the floating-point operation count of each generated body,
which the benchmark uses as the algorithmic work per quartet.

Usage: python gen_hgp.py OUTDIR
"""
from __future__ import annotations

import json
import os
import sys

PAIR_CLASSES = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
LNAME = "spd"


def cart(l):
    return [(lx, ly, l - lx - ly) for lx in range(l, -1, -1) for ly in range(l - lx, -1, -1)]


def ncart(l):
    return (l + 1) * (l + 2) // 2


def quartet_classes():
    out = []
    for X in range(len(PAIR_CLASSES)):
        for Y in range(X + 1):
            la, lb = PAIR_CLASSES[X]
            lc, ld = PAIR_CLASSES[Y]
            out.append((X, Y, la, lb, lc, ld))
    return out


def cls_name(la, lb, lc, ld):
    return f"{LNAME[la]}{LNAME[lb]}{LNAME[lc]}{LNAME[ld]}"


def sub(v, i, k=1):
    w = list(v)
    w[i] -= k
    return tuple(w)


def add(v, i, k=1):
    w = list(v)
    w[i] += k
    return tuple(w)


XYZ = "xyz"


class Code:
    def __init__(self, prefix):
        self.lines = []
        self.memo = {}
        self.n = 0
        self.prefix = prefix
        self.flops = 0

    def emit(self, expr, flops):
        name = f"{self.prefix}{self.n}"
        self.n += 1
        self.lines.append(f"const T {name} = {expr};")
        self.flops += flops
        return name


class VRR(Code):
    """Vertical recurrences for one class; nodes are [e0|f0]^(m)."""

    def __init__(self, L):
        super().__init__("v")
        self.L = L

    def node(self, e, f, m):
        key = (e, f, m)
        if key in self.memo:
            return self.memo[key]
        if any(x < 0 for x in e) or any(x < 0 for x in f):
            return None
        if sum(e) == 0 and sum(f) == 0:
            name = f"F[{m}]"
            self.memo[key] = name
            return name
        if sum(f) == 0:
            name = self._bra(e, m)
        else:
            name = self._ket(e, f, m)
        self.memo[key] = name
        return name

    def _missing(self, key, seen):
        """Nodes that computing `key` would add (upper bound, no emission)."""
        if key in self.memo or key in seen:
            return 0
        e, f, m = key
        if any(x < 0 for x in e) or any(x < 0 for x in f) or (sum(e) == 0 and sum(f) == 0):
            return 0
        seen.add(key)
        if sum(f) == 0:
            i = next(k for k in range(3) if e[k] > 0)
            e1 = sub(e, i)
            ks = [(e1, f, m), (e1, f, m + 1), (sub(e1, i), f, m), (sub(e1, i), f, m + 1)]
        else:
            i = next(k for k in range(3) if f[k] > 0)
            f1 = sub(f, i)
            ks = [(e, f1, m), (e, f1, m + 1), (e, sub(f1, i), m), (e, sub(f1, i), m + 1),
                  (sub(e, i), f1, m + 1)]
        return 1 + sum(self._missing(k, seen) for k in ks)

    def accumulate(self, outputs, greedy=False):
        """Emit acc[t] += [e0|f0]^(0) for outputs [(t, e, f)], each add right after
        its value is available; with `greedy` the next output is the one that
        needs the fewest new nodes."""
        todo = list(outputs)
        while todo:
            j = 0
            if greedy:
                j = min(range(len(todo)),
                        key=lambda u: (self._missing((todo[u][1], todo[u][2], 0), set()), u))
            t, e, f = todo.pop(j)
            v = self.node(e, f, 0)
            self.lines.append(f"acc[{t}] += {v};")
        return len(outputs)

    def _pick(self, cands, children):
        best, best_cost = None, None
        for i in cands:
            cost = sum(1 for k in children(i) if k is not None and k not in self.memo)
            if best is None or cost < best_cost:
                best, best_cost = i, cost
        return best

    def _bra(self, e, m):
        f0 = (0, 0, 0)
        cands = [i for i in range(3) if e[i] > 0]

        def ch(i):
            e1 = sub(e, i)
            ks = [(e1, f0, m), (e1, f0, m + 1)]
            if e1[i] > 0:
                ks += [(sub(e1, i), f0, m), (sub(e1, i), f0, m + 1)]
            return ks

        i = self._pick(cands, ch)
        e1 = sub(e, i)
        a = self.node(e1, f0, m)
        b = self.node(e1, f0, m + 1)
        terms = [f"PA{XYZ[i]} * {a}", f"WP{XYZ[i]} * {b}"]
        fl = 3
        if e1[i] > 0:
            c = self.node(sub(e1, i), f0, m)
            d = self.node(sub(e1, i), f0, m + 1)
            k = e1[i]
            terms.append(f"T({k}) * (oo2p * {c} - oo2p_rp * {d})" if k > 1 else
                         f"(oo2p * {c} - oo2p_rp * {d})")
            fl += 4 + (1 if k > 1 else 0)
        return self.emit(" + ".join(terms), fl)

    def _ket(self, e, f, m):
        cands = [i for i in range(3) if f[i] > 0]

        def ch(i):
            f1 = sub(f, i)
            ks = [(e, f1, m), (e, f1, m + 1)]
            if f1[i] > 0:
                ks += [(e, sub(f1, i), m), (e, sub(f1, i), m + 1)]
            if e[i] > 0:
                ks += [(sub(e, i), f1, m + 1)]
            return ks

        i = self._pick(cands, ch)
        f1 = sub(f, i)
        a = self.node(e, f1, m)
        b = self.node(e, f1, m + 1)
        terms = [f"QC{XYZ[i]} * {a}", f"WQ{XYZ[i]} * {b}"]
        fl = 3
        if f1[i] > 0:
            c = self.node(e, sub(f1, i), m)
            d = self.node(e, sub(f1, i), m + 1)
            k = f1[i]
            terms.append(f"T({k}) * (oo2q * {c} - oo2q_rq * {d})" if k > 1 else
                         f"(oo2q * {c} - oo2q_rq * {d})")
            fl += 4 + (1 if k > 1 else 0)
        if e[i] > 0:
            g = self.node(sub(e, i), f1, m + 1)
            k = e[i]
            terms.append(f"T({k}) * oo2pq * {g}" if k > 1 else f"oo2pq * {g}")
            fl += 2 + (1 if k > 1 else 0)
        return self.emit(" + ".join(terms), fl)


def max_live(lines):
    """Largest number of recurrence temporaries alive at once in emitted order."""
    import re
    defs, last = {}, {}
    for n, ln in enumerate(lines):
        m = re.match(r"const T (\w+) = (.*);", ln)
        rhs = m.group(2) if m else ln
        for u in re.findall(r"\bv\d+\b", rhs):
            last[u] = n
        if m:
            defs[m.group(1)] = n
    ev = [0] * (len(lines) + 2)
    for v, d in defs.items():
        ev[d] += 1
        ev[last.get(v, d) + 1] -= 1
    cur = best = 0
    for x in ev:
        cur += x
        best = max(best, cur)
    return best


def build_vrr(L, outputs):
    """Straight-line recurrence code for the accumulator outputs [(t, e, f)]:
    of a few output orders, the one with the fewest live temporaries (register
    pressure of FP64 values on a 512-register file decides occupancy)."""
    orders = [list(outputs), sorted(outputs, key=lambda o: (o[2], o[1]))]
    best = None
    for greedy in (False, True):
        for order in orders:
            v = VRR(L)
            v.accumulate(order, greedy)
            score = (max_live(v.lines), v.flops)
            if best is None or score < best[0]:
                best = (score, v)
    return best[1]


def e_set(la, lb):
    return [c for l in range(la, la + lb + 1) for c in cart(l)]


class HRR(Code):
    """Horizontal recurrences on contracted [e0|f0]; nodes are (a b|c d)."""

    def __init__(self, la, lb, lc, ld):
        super().__init__("h")
        self.E = {c: i for i, c in enumerate(e_set(la, lb))}
        self.Fs = {c: i for i, c in enumerate(e_set(lc, ld))}
        self.nf = len(self.Fs)

    def node(self, a, b, c, d):
        key = (a, b, c, d)
        if key in self.memo:
            return self.memo[key]
        if sum(d) > 0:
            i = next(k for k in range(3) if d[k] > 0)
            x = self.node(a, b, add(c, i), sub(d, i))
            y = self.node(a, b, c, sub(d, i))
            name = self.emit(f"{x} + CD{XYZ[i]} * {y}", 2)
        elif sum(b) > 0:
            i = next(k for k in range(3) if b[k] > 0)
            x = self.node(add(a, i), sub(b, i), c, d)
            y = self.node(a, sub(b, i), c, d)
            name = self.emit(f"{x} + AB{XYZ[i]} * {y}", 2)
        else:
            name = f"acc[{self.E[a] * self.nf + self.Fs[c]}]"
        self.memo[key] = name
        return name


# Wavefronts per SIMD each class kernel is compiled for, per precision (FP64 / FP32
# value size in bytes); classes not listed take 1 (all 512 registers of a lane).
# JK_WAVES_OVERRIDE="kind:size:waves,..." (kind = single or split) overrides the
# listed kernels of one precision, for measurements.
# (Measured on gfx950 at 1080 functions: with the digestion in sweeps, two
# wavefronts per SIMD make the FP32 kernels of these classes 20-35 % faster; the
# FP64 ones, which spill at that budget, lose.)
CLASS_WAVES = {(name, 4): 2 for name in ("pppp", "dspp", "dsds", "dpps", "dpds", "ddps")}
# FP32 multi-pass kernels at two wavefronts per SIMD (256 registers; measured on
# gfx950 at 1080 functions: (dp|dp) 134 -> 100 ms, (dd|pp) 61 -> 53 ms, (dd|dd)
# 15 -> 13 ms; (dd|ds) and (dd|dp), which spill more at that budget, lose).
CLASS_WAVES.update({(name, 4): 2 for name in ("dpdp_f32", "ddpp_f32", "dddd_f32")})
# FP64 multi-pass (dp|pp) and (dp|dp) at two wavefronts per SIMD (measured on gfx950
# at 1080 functions, FP64 build: 381 -> 365 ms and 265 -> 234 ms; the other FP64
# multi-pass classes lose, up to 2.2x for (dd|ds)).
CLASS_WAVES.update({(name, 8): 2 for name in ("dppp", "dpdp")})


def class_waves(name, size, split=False):
    ov = os.environ.get("JK_WAVES_OVERRIDE", "")
    for item in filter(None, ov.split(",")):
        kind, sz, w = item.split(":")
        if int(sz) == size and kind == ("split" if split else "single"):
            return int(w)
    return CLASS_WAVES.get((name, size), 1)


def lanes_for(L, split):
    """Most lanes that share one shell quartet: light classes 1, mid classes 4, heavy 16."""
    if split:
        return 16
    return 1 if L <= 2 else 4


LDS_MAX_L = 3   # single-pass classes up to this order read the Boys rows from LDS
ROWS_BLOCK = 512   # threads of the light-class kernel that keeps the bra's K rows in LDS
# Light classes and precisions that use the rows kernel ("name:size"); JK_ROWS_OVERRIDE
# = "all" or "none" for measurements.
# (Measured on gfx950 at 1080 functions: the row buffer halves the time of the
# atomic-bound FP32 kernels of the lightest classes; the FP64 kernels of most light
# classes are bound by arithmetic and run faster as 1024-thread workgroups without it.)
ROWS_CLASSES = {"ssss:8", "ppps:8", "dsps:8", "ssss:4", "psss:4", "psps:4", "ppss:4", "dsss:4"}


def uses_rows(name, size):
    ov = os.environ.get("JK_ROWS_OVERRIDE", "")
    if ov == "none":
        return False
    if ov == "all" or ROWS_CLASSES is None:
        return True
    return f"{name}:{size}" in ROWS_CLASSES


# Of those, the classes that also take the row buffer with several densities (one
# launch per density, the integrals recomputed each time): FP32 classes whose
# integrals cost less than the per-density scatter of the other kernel.  (Measured
# on gfx950 at 1800 functions and 10 densities: (ss|ss) 2.76 -> 1.24 s, (ps|ss)
# 8.65 -> 5.36 s, (ps|ps) 8.77 -> 7.47 s; (pp|ss) and (ds|ss) lose 9-12 %.)
ROWS_MULTI_CLASSES = {"ssss:4", "psss:4", "psps:4"}


def rows_call(name, t, att=False):
    size = 8 if t == "double" else 4
    if not uses_rows(name, size):
        return "false"
    multi = "true" if f"{name}:{size}" in ROWS_MULTI_CLASSES else "false"
    return f"launch_rows<Cls_{name}, {t}, {ROWS_BLOCK}, {multi}, {'true' if att else 'false'}>(a, s)"

# Single-pass classes whose kernels digest in five sweeps (one J/K block each).
# JK_SWEEPS_OVERRIDE=1 turns sweeps on for every class above LDS_MAX_L, for
# measurements.
# (Measured on gfx950 at 1080 functions: 10-40 % faster for these classes in both
# precisions, no change for the others.)
SWEEP_CLASSES = {"pppp", "dspp", "dsds", "dpps", "dpds", "ddps"}


def uses_sweeps(sname):
    if os.environ.get("JK_SWEEPS_OVERRIDE") == "1":
        L = sum("spd".index(ch) for ch in sname[:4])
        return L > LDS_MAX_L
    return sname in SWEEP_CLASSES or sname.endswith("_f32")


def uses_lds(L, split):
    return not split and L <= LDS_MAX_L


def lane_options(L, split):
    """Lane counts a class is compiled for; the host picks one per launch.  (One
    lane per quartet also for (dd|dp) and (dd|dd) since their workspace addresses
    no longer spill: measured on gfx950 at 1080 functions, (dd|dp) FP64 194 -> 163 ms.)"""
    if split:
        return [1, 4, 16]
    return [1] if uses_lds(L, split) else [1, 4]


def gen_class(la, lb, lc, ld, suffix=""):
    L = la + lb + lc + ld
    name = cls_name(la, lb, lc, ld)
    sname = name + suffix   # struct Cls_<sname>
    E = e_set(la, lb)
    Fs = e_set(lc, ld)
    ne, nf = len(E), len(Fs)
    na, nb, nc, nd = ncart(la), ncart(lb), ncart(lc), ncart(ld)

    outs = [(ie * nf + jf, e, f) for ie, e in enumerate(E) for jf, f in enumerate(Fs)]
    vrr = build_vrr(L, outs)
    vrr_flops = vrr.flops + len(outs)

    hrr = HRR(la, lb, lc, ld)
    n_int = 0
    A, B, C, D = cart(la), cart(lb), cart(lc), cart(ld)
    for ia, a in enumerate(A):
        for ib, b in enumerate(B):
            for ic, c in enumerate(C):
                for id_, d in enumerate(D):
                    h = hrr.node(a, b, c, d)
                    n_int += 1
                    # digest each integral right after it is formed: few live values
                    hrr.lines.append(
                        f"{{ const double v = double({h}) * fq;"
                        f" jab[{ia * nb + ib}] += Dcd[{ic * nd + id_}] * v;"
                        f" jcd[{ic * nd + id_}] += Dab[{ia * nb + ib}] * v;"
                        f" kac[{ia * nc + ic}] += Dbd[{ib * nd + id_}] * v;"
                        f" kad[{ia * nd + id_}] += Dbc[{ib * nc + ic}] * v;"
                        f" kbc[{ib * nc + ic}] += Dad[{ia * nd + id_}] * v;"
                        f" kbd[{ib * nd + id_}] += Dac[{ia * nc + ic}] * v; }}")
    hrr_flops = hrr.flops
    dig_flops = 13 * n_int

    # The same horizontal recurrences split into five sweeps, each digesting into
    # one block (J: jab and jcd; then kac, kad, kbc, kbd): a sweep holds only its
    # own D block and accumulators live, at the price of recomputing the HRR.
    sweeps = []
    blocks = [("j", None), ("kac", ("Dbd", "ib * nd + id_", "ia * nc + ic")),
              ("kad", ("Dbc", "ib * nc + ic", "ia * nd + id_")),
              ("kbc", ("Dad", "ia * nd + id_", "ib * nc + ic")),
              ("kbd", ("Dac", "ia * nc + ic", "ib * nd + id_"))]
    for bname, spec in blocks:
        hs = HRR(la, lb, lc, ld)
        for ia, a in enumerate(A):
            for ib, b in enumerate(B):
                for ic, c in enumerate(C):
                    for id_, d in enumerate(D):
                        h = hs.node(a, b, c, d)
                        if spec is None:
                            hs.lines.append(
                                f"{{ const double v = double({h}) * fq;"
                                f" jab[{ia * nb + ib}] += Dcd[{ic * nd + id_}] * v;"
                                f" jcd[{ic * nd + id_}] += Dab[{ia * nb + ib}] * v; }}")
                        else:
                            dn, di, oi = spec
                            env = dict(ia=ia, ib=ib, ic=ic, id_=id_, na=na, nb=nb, nc=nc, nd=nd)
                            hs.lines.append(f"{bname}[{eval(oi, env)}] += {dn}[{eval(di, env)}] * "
                                            f"(double({h}) * fq);")
        sweeps.append((bname, hs.lines))

    diag_code = None
    if (la, lb) == (lc, ld):
        dh = HRR(la, lb, lc, ld)
        out = []
        for ia, a in enumerate(A):
            for ib, b in enumerate(B):
                h = dh.node(a, b, a, b)
                out.append(f"mx = fmax(mx, double({h}));")
        diag_code = (dh.lines, out)

    s = []
    s.append(f"// class ({LNAME[la]}{LNAME[lb]}|{LNAME[lc]}{LNAME[ld]}): L = {L}, "
             f"{ne}x{nf} contracted [e0|f0], {na * nb * nc * nd} integrals")
    s.append(f"struct Cls_{sname} {{")
    s.append(f"  static constexpr int LA = {la}, LB = {lb}, LC = {lc}, LD = {ld}, L = {L};")
    s.append(f"  static constexpr int NA = {na}, NB = {nb}, NC = {nc}, ND = {nd};")
    s.append(f"  static constexpr int NE = {ne}, NF = {nf}, NACC = {ne * nf};")
    s.append(f"  static constexpr int GMAX = {lanes_for(L, False)};  // most lanes per shell quartet")
    s.append(f"  static constexpr int WAVES64 = {class_waves(sname, 8)}, WAVES32 = {class_waves(sname, 4)};")
    s.append(f"  static constexpr int VRR_FLOPS = {vrr_flops}, HRR_FLOPS = {hrr_flops}, "
             f"DIGEST_FLOPS = {dig_flops};")
    s.append("  template <typename T>")
    s.append("  __device__ __forceinline__ static void vrr(const T* __restrict__ F, const VrrCoef<T>& c,"
             " T* __restrict__ acc) {")
    s.append("    const T PAx = c.PAx, PAy = c.PAy, PAz = c.PAz, WPx = c.WPx, WPy = c.WPy, WPz = c.WPz;")
    s.append("    const T QCx = c.QCx, QCy = c.QCy, QCz = c.QCz, WQx = c.WQx, WQy = c.WQy, WQz = c.WQz;")
    s.append("    const T oo2p = c.oo2p, oo2p_rp = c.oo2p_rp, oo2q = c.oo2q, oo2q_rq = c.oo2q_rq, "
             "oo2pq = c.oo2pq;")
    s.append("    (void)PAx; (void)PAy; (void)PAz; (void)WPx; (void)WPy; (void)WPz; (void)QCx; (void)QCy;"
             " (void)QCz; (void)WQx; (void)WQy; (void)WQz; (void)oo2p; (void)oo2p_rp; (void)oo2q;"
             " (void)oo2q_rq; (void)oo2pq;")
    s += ["    " + x for x in vrr.lines]
    s.append("  }")
    s.append("  template <typename T>")
    s.append("  __device__ __forceinline__ static void hrr_digest(const T* __restrict__ acc, T ABx, T ABy, T ABz,"
             " T CDx, T CDy, T CDz, double fq, const double* Dab, const double* Dcd,"
             " const double* Dac, const double* Dad, const double* Dbc, const double* Dbd,"
             " double* jab, double* jcd, double* kac, double* kad, double* kbc, double* kbd) {")
    s.append("    (void)ABx; (void)ABy; (void)ABz; (void)CDx; (void)CDy; (void)CDz;")
    s += ["    " + x for x in hrr.lines]
    s.append("  }")
    s.append(f"  static constexpr int SWEEPS = {1 if uses_sweeps(sname) else 0};  // digestion in five sweeps")
    sig = {"j": "const double* Dab, const double* Dcd, double* jab, double* jcd",
           "kac": "const double* Dbd, double* kac", "kad": "const double* Dbc, double* kad",
           "kbc": "const double* Dad, double* kbc", "kbd": "const double* Dac, double* kbd"}
    for bname, lines in sweeps:
        s.append("  template <typename T>")
        s.append(f"  __device__ __forceinline__ static void digest_{bname}(const T* __restrict__ acc, T ABx, T ABy,"
                 f" T ABz, T CDx, T CDy, T CDz, double fq, {sig[bname]}) {{")
        s.append("    (void)ABx; (void)ABy; (void)ABz; (void)CDx; (void)CDy; (void)CDz;")
        s += ["    " + x for x in lines]
        s.append("  }")
    if diag_code is not None:
        s.append("  template <typename T>")
        s.append("  __device__ __forceinline__ static double diag_max(const T* __restrict__ acc, T ABx, T ABy,"
                 " T ABz) {")
        s.append("    const T CDx = ABx, CDy = ABy, CDz = ABz;")
        s.append("    (void)CDx; (void)CDy; (void)CDz; (void)ABx; (void)ABy; (void)ABz;")
        s.append("    double mx = 0.0;")
        s += ["    " + x for x in diag_code[0]]
        s += ["    " + x for x in diag_code[1]]
        s.append("    return mx;")
        s.append("  }")
    s.append("};")
    info = dict(name=name, sname=sname, la=la, lb=lb, lc=lc, ld=ld, L=L, nacc=ne * nf,
                nint=na * nb * nc * nd, vrr_flops=vrr_flops, hrr_flops=hrr_flops,
                digest_flops=dig_flops, vrr_nodes=vrr.n, hrr_nodes=hrr.n, nf=nf,
                vrr_flops_alg=vrr_flops, lanes=lanes_for(L, False),
                lane_options=lane_options(L, False), lds=uses_lds(L, False),
                lds_block=1024 if L <= 2 else 512)
    return "\n".join(s) + "\n", info


# Classes with more contracted accumulators than SPLIT_NACC use the multi-pass
# form; a pass holds at most PASS_ACC accumulators: a block of consecutive bra
# components e with every ket component f.  Blocks of e share less of the
# recurrence tree than blocks of f do (each [e0|f0] is reached from lower f at
# the same e), so splitting along e repeats less work and keeps fewer values
# alive: for (dd|dp) 9.6k instead of 16.7k recurrence flops per primitive
# quartet over all passes, with at most 50 instead of 105 live temporaries.
# (Measured on gfx950: single-pass classes up to about 100 FP64 accumulators
# beat their multi-pass form.)
SPLIT_NACC = 100
PASS_ACC = 64


def pass_chunks(ne, nf, cap=None):
    """Pass j covers bra components chunks[j] (with all nf ket components)."""
    cap = cap or PASS_ACC
    npass = -(-ne // max(1, cap // nf))      # fewest passes of whole bra components
    chunk = -(-ne // npass)                  # spread evenly over them
    return [list(range(i, min(i + chunk, ne))) for i in range(0, ne, chunk)]


# Larger passes where they still fit: up to PASS_ACC_WIDE accumulators when those
# plus the pass's most live recurrence temporaries stay within PASS_LIVE FP64
# values (2 VGPRs each).  (Measured on gfx950: (dp|pp) and (dd|ds) gain 6-9 %
# from fewer passes; (dp|dp) and (dd|dp), above the bound, lose.)
PASS_ACC_WIDE = 96
PASS_LIVE = 140

# FP32 values take one VGPR instead of two, so the FP32 kernels of these classes
# get their own layout: single-pass up to SPLIT_NACC32 accumulators (digestion in
# sweeps), else passes twice the FP64 sizes.
SPLIT_NACC32 = 160
PASS_ACC32, PASS_ACC_WIDE32, PASS_LIVE32 = 128, 192, 280


def split_chunks(L, E, Fs, pass_acc=None, pass_acc_wide=None, pass_live=None):
    pass_acc = pass_acc or PASS_ACC
    wide = pass_chunks(len(E), len(Fs), pass_acc_wide or PASS_ACC_WIDE)
    worst = 0
    for ch in wide:
        outs = [(ii * len(Fs) + jf, E[ie], f) for ii, ie in enumerate(ch) for jf, f in enumerate(Fs)]
        worst = max(worst, len(outs) + max_live(build_vrr(L, outs).lines))
    return wide if worst <= (pass_live or PASS_LIVE) else pass_chunks(len(E), len(Fs), pass_acc)


class KetHRR(Code):
    """|c d) from |f 0) for one bra component: nodes keyed (c, d)."""

    def __init__(self, lc, ld):
        super().__init__("k")
        self.Fs = {c: i for i, c in enumerate(e_set(lc, ld))}

    def node(self, c, d):
        key = (c, d)
        if key in self.memo:
            return self.memo[key]
        if sum(d) > 0:
            i = next(k for k in range(3) if d[k] > 0)
            x = self.node(add(c, i), sub(d, i))
            y = self.node(c, sub(d, i))
            name = self.emit(f"{x} + CD{XYZ[i]} * {y}", 2)
        else:
            name = f"f[{self.Fs[c]}]"
        self.memo[key] = name
        return name


class BraHRR(Code):
    """(a b| from (e 0| for one ket component: nodes keyed (a, b)."""

    def __init__(self, la, lb):
        super().__init__("b")
        self.E = {c: i for i, c in enumerate(e_set(la, lb))}

    def node(self, a, b):
        key = (a, b)
        if key in self.memo:
            return self.memo[key]
        if sum(b) > 0:
            i = next(k for k in range(3) if b[k] > 0)
            x = self.node(add(a, i), sub(b, i))
            y = self.node(a, sub(b, i))
            name = self.emit(f"{x} + AB{XYZ[i]} * {y}", 2)
        else:
            name = f"e[{self.E[a]}]"
        self.memo[key] = name
        return name


VRR_PROLOGUE = [
    "const T PAx = c.PAx, PAy = c.PAy, PAz = c.PAz, WPx = c.WPx, WPy = c.WPy, WPz = c.WPz;",
    "const T QCx = c.QCx, QCy = c.QCy, QCz = c.QCz, WQx = c.WQx, WQy = c.WQy, WQz = c.WQz;",
    "const T oo2p = c.oo2p, oo2p_rp = c.oo2p_rp, oo2q = c.oo2q, oo2q_rq = c.oo2q_rq, oo2pq = c.oo2pq;",
    "(void)PAx; (void)PAy; (void)PAz; (void)WPx; (void)WPy; (void)WPz; (void)QCx; (void)QCy;"
    " (void)QCz; (void)WQx; (void)WQy; (void)WQz; (void)oo2p; (void)oo2p_rp; (void)oo2q;"
    " (void)oo2q_rq; (void)oo2pq;",
]


def gen_split_class(la, lb, lc, ld, suffix="", pass_acc=None, pass_acc_wide=None,
                    pass_live=None):
    """Multi-pass form: each pass accumulates (a block of E) x F in registers."""
    L = la + lb + lc + ld
    name = cls_name(la, lb, lc, ld)
    sname = name + suffix   # struct Cls_<sname>
    E = e_set(la, lb)
    Fs = e_set(lc, ld)
    ne, nf = len(E), len(Fs)
    na, nb, nc, nd = ncart(la), ncart(lb), ncart(lc), ncart(ld)
    chunks = split_chunks(L, E, Fs, pass_acc, pass_acc_wide, pass_live)
    chunk = len(chunks[0])
    s = []
    s.append(f"// class ({LNAME[la]}{LNAME[lb]}|{LNAME[lc]}{LNAME[ld]}): L = {L}, "
             f"{ne}x{nf} contracted [e0|f0] built in {len(chunks)} passes of "
             f"<= {len(chunks[0])} bra components, {na * nb * nc * nd} integrals")
    s.append(f"struct Cls_{sname} {{")
    s.append(f"  static constexpr int LA = {la}, LB = {lb}, LC = {lc}, LD = {ld}, L = {L};")
    s.append(f"  static constexpr int NA = {na}, NB = {nb}, NC = {nc}, ND = {nd};")
    s.append(f"  static constexpr int NE = {ne}, NF = {nf}, NACC = {ne * nf};")
    s.append(f"  static constexpr int NPASS = {len(chunks)}, ECHUNK = {chunk};")
    s.append(f"  static constexpr int GMAX = {lanes_for(L, True)};  // most lanes per shell quartet")
    s.append(f"  static constexpr int WAVES64 = {class_waves(sname, 8, True)}, "
             f"WAVES32 = {class_waves(sname, 4, True)};")
    vrr_flops = 0
    for j, ch in enumerate(chunks):
        outs = [(ii * nf + jf, E[ie], f) for ii, ie in enumerate(ch) for jf, f in enumerate(Fs)]
        v = build_vrr(L, outs)
        lines = []
        vrr_flops += v.flops + len(outs)
        s.append("  template <typename T>")
        s.append(f"  __device__ __forceinline__ static void vrr_p{j}(const T* __restrict__ F, "
                 "const VrrCoef<T>& c, T* __restrict__ acc) {")
        s += ["    " + x for x in VRR_PROLOGUE]
        s += ["    " + x for x in v.lines]
        s += ["    " + x for x in lines]
        s.append("  }")
    s.append("  template <int J, typename T>")
    s.append("  __device__ __forceinline__ static void vrr_pass(const T* __restrict__ F, "
             "const VrrCoef<T>& c, T* __restrict__ acc) {")
    for j in range(len(chunks)):
        kw = "if" if j == 0 else "else if"
        s.append(f"    {kw} constexpr (J == {j}) vrr_p{j}<T>(F, c, acc);")
    s.append("  }")
    s.append("  template <int J> struct Pass;")
    kh = KetHRR(lc, ld)
    outs = []
    for ic, cc in enumerate(cart(lc)):
        for id_, dd in enumerate(cart(ld)):
            outs.append(f"out[{ic * nd + id_}] = {kh.node(cc, dd)};")
    s.append("  template <typename T>")
    s.append("  __device__ __forceinline__ static void ket_hrr(const T* __restrict__ f, T CDx, T CDy, "
             "T CDz, T* __restrict__ out) {")
    s.append("    (void)CDx; (void)CDy; (void)CDz;")
    s += ["    " + x for x in kh.lines]
    s += ["    " + x for x in outs]
    s.append("  }")
    bh = BraHRR(la, lb)
    outs = []
    for ia, aa in enumerate(cart(la)):
        for ib, bb in enumerate(cart(lb)):
            outs.append(f"out[{ia * nb + ib}] = {bh.node(aa, bb)};")
    s.append("  template <typename T>")
    s.append("  __device__ __forceinline__ static void bra_hrr(const T* __restrict__ e, T ABx, T ABy, "
             "T ABz, T* __restrict__ out) {")
    s.append("    (void)ABx; (void)ABy; (void)ABz;")
    s += ["    " + x for x in bh.lines]
    s += ["    " + x for x in outs]
    s.append("  }")
    hrr_flops = kh.flops * ne + bh.flops * nc * nd
    dig_flops = 13 * na * nb * nc * nd
    s.append(f"  static constexpr int VRR_FLOPS = {vrr_flops}, HRR_FLOPS = {hrr_flops}, "
             f"DIGEST_FLOPS = {dig_flops};")
    s.append("};")
    for j, ch in enumerate(chunks):
        s.append(f"template <> struct Cls_{sname}::Pass<{j}> {{ static constexpr int E0 = {ch[0]}, "
                 f"NE = {len(ch)}; }};")
    one = VRR(L)
    for e in E:
        for f in Fs:
            one.node(e, f, 0)
    info = dict(name=name, sname=sname, la=la, lb=lb, lc=lc, ld=ld, L=L, nacc=ne * nf,
                nint=na * nb * nc * nd, vrr_flops=vrr_flops, hrr_flops=hrr_flops,
                digest_flops=dig_flops, npass=len(chunks), split=True, nf=nf,
                vrr_flops_alg=one.flops + ne * nf, lanes=lanes_for(L, True),
                lane_options=lane_options(L, True))
    return "\n".join(s) + "\n", info


PAIR_NAME = {pc: LNAME[pc[0]] + LNAME[pc[1]] for pc in PAIR_CLASSES}


def wrapper(info, att=False):
    """Launch function of one class: launch_eri_<name> for the 1/r12 kernels, or
    (att) launch_eri_att_<name> for those of erf(omega r12)/r12, which take the
    same launch shapes; each goes to a translation unit of its own."""
    n = info["name"]
    fn = f"launch_eri_att_{n}" if att else f"launch_eri_{n}"
    ta = ", true" if att else ""
    kern = "eri_jk_split_kernel" if info["split"] else "eri_jk_kernel"
    skern = "schwarz_split_kernel" if info["split"] else "schwarz_kernel"
    i32 = info.get("f32", info)   # FP32 layout (the class itself unless it has its own)
    n32 = i32["sname"]
    kern32 = "eri_jk_split_kernel" if i32["split"] else "eri_jk_kernel"
    w = [f"// generated by gen_hgp.py -- do not edit",
         '#include "jk_classes.hpp"',
         "namespace jk {",
         f'#include "cls_{n}.inc"',
         f"void {fn}(const EriLaunch& a, int fp32, hipStream_t s) {{",
         *([f"  // the bra's exchange rows in LDS, where they fit",
            f"  if (a.rows && (fp32 ? {rows_call(n, 'float', att)}",
            f"                      : {rows_call(n, 'double', att)})) return;",
            f"  // Boys rows staged in LDS; as many workgroups as fit on the device claim the items",
            f"  constexpr int NT = {info.get('lds_block', 0)};",
            f"  static int per_cu[2] = {{0, 0}};",
            f"  if (!per_cu[fp32]) {{",
            f"    int nb = 0;",
            f"    if (fp32) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&eri_jk_lds_kernel<Cls_{n}, float, NT{ta}>), NT, 0);",
            f"    else (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&eri_jk_lds_kernel<Cls_{n}, double, NT{ta}>), NT, 0);",
            f"    per_cu[fp32] = nb > 0 ? nb : 1;",
            f"  }}",
            f"  const dim3 lgrid(std::min((a.nitems + NT / kWave - 1) / (NT / kWave), per_cu[fp32] * a.num_cu));",
            f"  if (fp32) launch_kernel(&eri_jk_lds_kernel<Cls_{n}, float, NT{ta}>, lgrid, dim3(NT), 0, s, a.dry != 0, a);",
            f"  else launch_kernel(&eri_jk_lds_kernel<Cls_{n}, double, NT{ta}>, lgrid, dim3(NT), 0, s, a.dry != 0, a);",
            "}"] if info.get("lds") else []),
         *([] if info.get("lds") else [
         "  const dim3 block(kBlock);",
         "  if (fp32) {",
         "    const int waves = " + ("a.nwaves" if i32["split"] else "a.nitems") + ";",
         "    const dim3 grid((waves + kWavesPerBlock - 1) / kWavesPerBlock);",
         *[ln for g_ in i32["lane_options"] for ln in (
             f"    {'if' if g_ == i32['lane_options'][0] else 'else if'} (a.lanes == {g_} || "
             f"{'true' if g_ == i32['lane_options'][-1] else 'false'})",
             f"      launch_kernel(&{kern32}<Cls_{n32}, float, {g_}{ta}>, grid, block, 0, s, a.dry != 0, a);")],
         "    return;",
         "  }",
         "  const int waves = " + ("a.nwaves" if info["split"] else "a.nitems") + ";",
         "  const dim3 grid((waves + kWavesPerBlock - 1) / kWavesPerBlock);",
         *[ln for g_ in info["lane_options"] for ln in (
             f"  {'if' if g_ == info['lane_options'][0] else 'else if'} (a.lanes == {g_} || "
             f"{'true' if g_ == info['lane_options'][-1] else 'false'})",
             f"    launch_kernel(&{kern}<Cls_{n}, double, {g_}{ta}>, grid, block, 0, s, a.dry != 0, a);")],
         "}"])]
    if info["bra_class"] == info["ket_class"] and not att:   # screening bounds: 1/r12
        w += [f"void launch_schwarz_{n}(const EriLaunch& a, double* Q, hipStream_t s) {{",
              (f"  launch_kernel(&{skern}<Cls_{n}>, dim3((a.nwaves + kWavesPerBlock - 1) / kWavesPerBlock),"
               " dim3(kBlock), 0, s, false, a, Q);") if info["split"] else
              (f"  launch_kernel(&{skern}<Cls_{n}>, dim3((a.bra.n * Cls_{n}::GMAX + kBlock - 1) / kBlock),"
               " dim3(kBlock), 0, s, false, a, Q);"),
              "}"]
    w.append("}  // namespace jk")
    return "\n".join(w) + "\n"


def table(infos):
    t = ["// generated by gen_hgp.py -- do not edit", '#include "jk_classes.hpp"', "namespace jk {"]
    for i in infos:
        t.append(f"void launch_eri_{i['name']}(const EriLaunch&, int, hipStream_t);")
        t.append(f"void launch_eri_att_{i['name']}(const EriLaunch&, int, hipStream_t);")
        if i["bra_class"] == i["ket_class"]:
            t.append(f"void launch_schwarz_{i['name']}(const EriLaunch&, double*, hipStream_t);")
    t.append("void launch_eri(int cls, int fp32, const EriLaunch& a, hipStream_t s) {")
    t.append("  switch (cls) {")
    for q, i in enumerate(infos):
        t.append(f"    case {q}: if (a.att) launch_eri_att_{i['name']}(a, fp32, s);"
                 f" else launch_eri_{i['name']}(a, fp32, s); break;")
    t.append("    default: break;")
    t.append("  }")
    t.append("}")
    t.append("// relative work per primitive quartet of each class (generated operation counts)")
    t.append("double class_cost(int cls, int grad) {")
    t.append("  static const double e[21] = {" + ", ".join(
        f"{i.get('vrr_flops_alg', i['vrr_flops']) + 71 + 4 * i['L'] + (i['hrr_flops'] + i['digest_flops']) / 81.0:.1f}"
        for i in infos) + "};")
    t.append("  static const double g[21] = {" + ", ".join(
        f"{3.0 * (i.get('vrr_flops_alg', i['vrr_flops']) + 71 + 4 * i['L']):.1f}" for i in infos) + "};")
    t.append("  if (cls < 0 || cls >= 21) return 1.0;")
    t.append("  return grad ? g[cls] : e[cls];")
    t.append("}")
    def wsb(i, tb):
        ncd = (i["lc"] + 1) * (i["lc"] + 2) // 2 * ((i["ld"] + 1) * (i["ld"] + 2) // 2)
        na = (i["la"] + 1) * (i["la"] + 2) // 2
        nb = (i["lb"] + 1) * (i["lb"] + 2) // 2
        nc = (i["lc"] + 1) * (i["lc"] + 2) // 2
        nd = (i["ld"] + 1) * (i["ld"] + 2) // 2
        ne = i["nacc"] // i["nf"]
        # per quartet slot: T values and the J_cd block; per lane: K partial blocks
        return ((i["nacc"] + ne * ncd) * tb + ncd * 8), 64 * (na * nc + na * nd + nb * nc + nb * nd) * 8
    t.append("// bytes of workspace per wavefront of the multi-pass classes with `lanes` lanes")
    t.append("// per quartet (0: not a multi-pass class); the kernels use split_wave_bytes")
    f32 = [i.get("f32", i) for i in infos]
    t.append("size_t split_ws_bytes(int cls, int fp32, int lanes) {")
    t.append("  static const size_t s64[21] = {" + ", ".join(str(wsb(i, 8)[0]) if i["split"] else "0" for i in infos) + "};")
    t.append("  static const size_t s32[21] = {" + ", ".join(str(wsb(i, 4)[0]) if i["split"] else "0" for i in f32) + "};")
    t.append("  static const size_t k64[21] = {" + ", ".join(str(wsb(i, 8)[1]) if i["split"] else "0" for i in infos) + "};")
    t.append("  static const size_t k32[21] = {" + ", ".join(str(wsb(i, 8)[1]) if i["split"] else "0" for i in f32) + "};")
    t.append("  if (cls < 0 || cls >= 21 || lanes < 1) return 0;")
    t.append("  const size_t k = fp32 ? k32[cls] : k64[cls];")
    t.append("  if (!k) return 0;")
    t.append("  return static_cast<size_t>(64 / lanes) * (fp32 ? s32[cls] : s64[cls]) + k;")
    t.append("}")
    t.append("// bytes per wavefront of the multi-pass Schwarz kernel of a diagonal class (FP64)")
    t.append("size_t split_schwarz_ws_bytes(int cls) {")
    t.append("  static const size_t w[21] = {" + ", ".join(
        str(64 * 8 * (i["nacc"] + (i["nacc"] // i["nf"]) * ((i["lc"] + 1) * (i["lc"] + 2) // 2) * ((i["ld"] + 1) * (i["ld"] + 2) // 2)))
        if i["split"] else "0" for i in infos) + "};")
    t.append("  return (cls >= 0 && cls < 21) ? w[cls] : 0;")
    t.append("}")
    t.append("// bit g set: the class has a kernel with g lanes per shell quartet")
    t.append("int class_lane_mask(int cls, int fp32) {")
    t.append("  static const int m[2][21] = {{" + ", ".join(str(sum(1 << g_ for g_ in i["lane_options"])) for i in infos) + "}, {"
             + ", ".join(str(sum(1 << g_ for g_ in i["lane_options"])) for i in f32) + "}};")
    t.append("  return (cls >= 0 && cls < 21) ? m[fp32 ? 1 : 0][cls] : 2;")
    t.append("}")
    t.append("int class_lanes(int cls, int fp32) {")
    t.append("  static const int g[2][21] = {{" + ", ".join(str(i["lanes"]) for i in infos) + "}, {"
             + ", ".join(str(i["lanes"]) for i in f32) + "}};")
    t.append("  return (cls >= 0 && cls < 21) ? g[fp32 ? 1 : 0][cls] : 1;")
    t.append("}")
    t.append("void launch_schwarz(int pair_class, const EriLaunch& a, double* Q, hipStream_t s) {")
    t.append("  switch (pair_class) {")
    for i in infos:
        if i["bra_class"] == i["ket_class"]:
            t.append(f"    case {i['bra_class']}: launch_schwarz_{i['name']}(a, Q, s); break;")
    t.append("    default: break;")
    t.append("  }")
    t.append("}")
    t.append("}  // namespace jk")
    return "\n".join(t) + "\n"


def write_if_changed(path, text):
    if not os.path.exists(path) or open(path).read() != text:
        with open(path, "w") as fh:
            fh.write(text)


def main(outdir):
    os.makedirs(outdir, exist_ok=True)
    infos = []
    for X, Y, la, lb, lc, ld in quartet_classes():
        ne, nf = len(e_set(la, lb)), len(e_set(lc, ld))
        if ne * nf > SPLIT_NACC:
            code, info = gen_split_class(la, lb, lc, ld)
            if ne * nf <= SPLIT_NACC32:
                code32, info32 = gen_class(la, lb, lc, ld, "_f32")
                info32["split"] = False
            else:
                code32, info32 = gen_split_class(la, lb, lc, ld, "_f32", PASS_ACC32, PASS_ACC_WIDE32,
                                                 PASS_LIVE32)
            info["f32"] = info32
            code += code32
        else:
            code, info = gen_class(la, lb, lc, ld)
            info["split"] = False
        info.update(bra_class=X, ket_class=Y)
        infos.append(info)
        name = info["name"]
        write_if_changed(os.path.join(outdir, f"cls_{name}.inc"),
                         "// generated by gen_hgp.py -- do not edit\n" + code)
        write_if_changed(os.path.join(outdir, f"cls_{name}.hip"), wrapper(info))
        write_if_changed(os.path.join(outdir, f"cls_{name}_att.hip"), wrapper(info, att=True))
    write_if_changed(os.path.join(outdir, "jk_classes_table.hip"), table(infos))
    write_if_changed(os.path.join(outdir, "classes.json"), json.dumps(infos, indent=1))
    return infos


if __name__ == "__main__":
    infos = main(sys.argv[1] if len(sys.argv) > 1 else "generated")
    for i in infos:
        print(f"{i['name']}: L={i['L']} acc={i['nacc']} ints={i['nint']} vrr_flops={i['vrr_flops']}"
              f" hrr={i['hrr_flops']} dig={i['digest_flops']}")
