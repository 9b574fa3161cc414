"""Write the tile-kernel instantiation units asm_{wq,ebe}_{f64,f32}.hip.

Each unit holds one switch from (degree p, points per element P) to the
kernel compiled for those compile-time sizes: WQ for p in 1..6 and
n_ref in 1..4 (P = 2 n_ref, Q = P (p+1) - 1 support nodes, first support node
1), EBE for p in 1..6 and G in 1..8 Gauss points (P = G, Q = G (p+1), first
support point 0).

Tile shapes: the sweep runs one work item per (node row, column strip), L x T/S
items with L = P (T - 1) + Q rows; the shape is chosen so that the items fill the
256 threads in one pass.  Fast form with n_ref = 1, p <= 4: 28 x 28 tiles with
7-column strips (236..252 items), and in FP64 from N = 4096 an instance compiled
for at least 4 waves per SIMD (FP32 reaches that occupancy anyway); p = 5, 6: 24 x 24 tiles, 6-column strips (228, 236
items).  FP64 fast form with n_ref = 3, 4: 16 x 16 tiles with 8-column
strips for p = 2..4 (measured at N = 1024: 1.1-1.5x faster than the scored shapes,
whose larger tiles held one or two workgroups per CU by LDS and registers; FP32
and n_ref = 2 gain nothing from it).  Otherwise the shape that function `shape`
scores best.
Run from this directory: python gen_instances.py
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))

HDR = '''// Instantiations of the tile kernel for {what} in {prec}: one kernel per
// (degree p, points per element P); written by gen_instances.py.
#include "tile_kernel.hpp"

namespace sgbem {{

hipError_t {fname}(int p, int P, const TileArgs &a, hipStream_t s, const KernelEvents *ev)
{{
    switch (p * 16 + P) {{
'''


SHAPES = [(32, 8), (28, 7), (24, 8), (24, 6), (21, 7), (20, 5), (16, 8), (16, 4), (12, 4), (8, 4)]


def shape(P, Q, ideal):
    """Tile edge T and strip width S for a sweep with P points per element and Q
    support points: maximise (fraction of 256 threads busy over the passes the
    L T/S items need) x (ideal kernel values per entry / values the tile
    evaluates per entry, halos included), L = P (T - 1) + Q."""
    def score(ts):
        T, S = ts
        L = P * (T - 1) + Q
        items = L * (T // S)
        passes = -(-items // 256)
        per_entry = L * (T // S) * (P * (S - 1) + Q) / (T * T)
        return items / (passes * 256) * ideal / per_entry
    return max(SHAPES, key=score)


def wq_cases():
    for p in range(1, 7):
        for R in range(1, 5):
            P = 2 * R
            if P == 2:
                T, S = (28, 7) if p <= 4 else (24, 6)
                yield p, P, P * (p + 1) - 1, 1, "true", T, S, (p <= 4)
            else:
                T, S = shape(P, P * (p + 1) - 1, P * P)
                yield p, P, P * (p + 1) - 1, 1, "true", T, S, False


def ebe_cases():
    for p in range(1, 7):
        for G in range(1, 9):
            T, S = shape(G, G * (p + 1), G * G)
            yield p, G, G * (p + 1), 0, "false", T, S, False


def main():
    for what, cases, tag in (("weighted-quadrature row assembly", wq_cases, "wq"),
                             ("the element-by-element far part", ebe_cases, "ebe")):
        for prec, real, suf in (("FP64", "double", "f64"), ("FP32", "float", "f32")):
            fname = f"launch_{tag}_{suf}"
            s = HDR.format(what=what, prec=prec, fname=fname)
            for (p, P, Q, S0, wq, T, S, big) in cases():
                if tag == "wq" and real == "double" and P >= 6 and 2 <= p <= 4:
                    T, S = 16, 8
                k = f"launch_tile<{P}, {Q}, {S0}, {wq}, {real}, {T}, {S}"
                if big and real == "double":
                    s += f"    case {p * 16 + P}: return a.N >= 4096 ? {k}, 4>(a, s, ev) : {k}>(a, s, ev);\n"
                elif big:
                    # FP32: bound the registers to >= 6 waves per SIMD (left alone, the compiler
                    # hoists the sweep's loads into 152 VGPRs; 56 VGPRs run 1.3x faster)
                    s += f"    case {p * 16 + P}: return {k}, 6>(a, s, ev);\n"
                else:
                    s += f"    case {p * 16 + P}: return {k}>(a, s, ev);\n"
            s += "    default: return hipErrorInvalidValue;\n    }\n}\n\n}  // namespace sgbem\n"
            with open(os.path.join(HERE, f"asm_{tag}_{suf}.hip"), "w") as f:
                f.write(s)


if __name__ == "__main__":
    main()
