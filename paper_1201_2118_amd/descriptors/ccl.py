"""Kernel descriptors -> HIP tile / halo / load / store code (build time).

The paper's kernel abstraction ("CaCUDA Kernel Abstraction") has three
parts: descriptors that declare a kernel's variables and their properties,
templates of optimised kernels, and a generator that parses the
descriptors with a parsing expression grammar and writes the boilerplate.
This module is that generator for gfx950: ``parse`` reads a descriptor file
(grammar below) into ``Kernel`` records, ``generate`` writes one HIP header
per kernel from the 3DBLOCK template, and ``build`` does both for a
directory.  The per-cell arithmetic is not generated: each kernel's body is
hand-written (``csrc/bodies/<name lower case>.h``) against the accessors the
header defines.

Grammar (parsing expression grammar; ``#`` starts a comment):

    file      <- (kernel)* EOF
    kernel    <- 'KERNEL' NAME attr* '{' (variable / parameter)* '}'
    variable  <- 'VARIABLE' attr* '{' names '}' STRING
    parameter <- 'PARAMETER' attr* '{' names '}' STRING
    attr      <- NAME '=' (STRING / WORD)
    names     <- NAME (',' NAME)*

Kernel attributes: TYPE (3DBLOCK or 3DSTREAM), STENCIL ("x-,x+,y-,y+,z-,z+"
halo cells, 0 or 1 each: the fields carry one ghost layer), TILE ("x,y,z"
cells per workgroup tile; x * y threads, x a multiple of 64, each thread
marching z cells).  Variable attributes: CACHED (YES: staged in LDS with the halo),
INTENT (IN, OUT, INOUT, SEPARATEINOUT), STORAGE (FIELD: the storage type of
the fields, FP64), OPTIONAL (YES: the group may be absent; a template flag).
Parameter attributes: SOURCE (VALUE: an FP64 kernel argument, CONTROL: the
field of the same name of the domain's control block, read on the device).

3DBLOCK, for tile (bx, by, bz) of a domain: every thread of the workgroup
loads the cached variables' box (tile plus halo) into LDS, x fastest (one
wave reads 64 consecutive x), with positions clamped to the padded array;
after one barrier thread (tx, ty) runs the body for the cells
(i0 + tx, j0 + ty, k0 + kz), kz = 0 .. z - 1, that are interior cells.

3DSTREAM, the same tile marched plane by plane: each cached variable lives
in a ring of z- + 1 + z+ LDS planes, each plane staged with its x / y halo;
while the body runs on plane k, every thread holds its share of plane
k + z+ + 1 in registers, and between two barriers it replaces plane k - z-
in the ring.  A cached value is loaded once per tile column instead of once
per box (the box's z halo is not re-read), and the next plane's loads are in
flight during the current plane's arithmetic.
"""
from __future__ import annotations

import os
import re
import sys
from dataclasses import dataclass, field

INTENTS = ("IN", "OUT", "INOUT", "SEPARATEINOUT")


class DescriptorError(ValueError):
    pass


@dataclass
class Variable:
    names: list
    group: str
    cached: bool = False
    intent: str = "IN"
    fp64: bool = False
    optional: bool = False
    line: int = 0


@dataclass
class Parameter:
    names: list
    group: str
    control: bool = False
    line: int = 0


@dataclass
class Kernel:
    name: str
    type: str = "3DBLOCK"
    stencil: tuple = (0, 0, 0, 0, 0, 0)
    tile: tuple = (64, 4, 4)
    variables: list = field(default_factory=list)
    parameters: list = field(default_factory=list)
    line: int = 0

    def all_vars(self):
        for v in self.variables:
            for n in v.names:
                yield n, v

    def optional_groups(self):
        return [v.group for v in self.variables if v.optional]


# ---- parser ------------------------------------------------------------------

_TOKEN = re.compile(r'(#[^\n]*)|("[^"\n]*")|([A-Za-z_][A-Za-z0-9_]*|[0-9][A-Za-z0-9_]*)|([{}=,])|(\s+)|(.)')


def _tokens(text):
    out = []
    for m in _TOKEN.finditer(text):
        comment, string, word, punct, space, bad = m.groups()
        line = text.count("\n", 0, m.start()) + 1
        if bad is not None:
            raise DescriptorError(f"line {line}: unexpected character {bad!r}")
        if string is not None:
            out.append(("STRING", string[1:-1], line))
        elif word is not None:
            out.append(("WORD", word, line))
        elif punct is not None:
            out.append((punct, punct, line))
    out.append(("EOF", "", text.count("\n") + 1))
    return out


class _Parser:
    def __init__(self, text):
        self.t = _tokens(text)
        self.i = 0

    def peek(self):
        return self.t[self.i]

    def take(self, kind, value=None, what=None):
        tok = self.t[self.i]
        if what:
            want = what
        elif value is not None:
            want = repr(value)
        elif kind == "WORD":
            want = "a name"
        else:
            want = repr(kind)
        if tok[0] != kind or (value is not None and tok[1] != value):
            raise DescriptorError(f"line {tok[2]}: expected {want}, found {tok[1]!r}")
        self.i += 1
        return tok

    def attrs(self):
        out = {}
        while self.peek()[0] == "WORD" and self.t[self.i + 1][0] == "=":
            name = self.take("WORD")[1].upper()
            self.take("=")
            tok = self.peek()
            if tok[0] not in ("STRING", "WORD"):
                raise DescriptorError(f"line {tok[2]}: attribute {name} needs a value")
            self.i += 1
            if name in out:
                raise DescriptorError(f"line {tok[2]}: attribute {name} given twice")
            out[name] = (tok[1], tok[2])
        return out

    def names(self):
        out = [self.take("WORD")[1]]
        while self.peek()[0] == ",":
            self.take(",")
            out.append(self.take("WORD")[1])
        return out

    def block(self, what):
        line = self.take("WORD", what)[2]
        attrs = self.attrs()
        self.take("{")
        names = self.names()
        self.take("}")
        group = self.take("STRING", what="a group name string")[1]
        return attrs, names, group, line

    def kernel(self):
        line = self.take("WORD", "KERNEL")[2]
        k = Kernel(name=self.take("WORD")[1], line=line)
        for key, (val, ln) in self.attrs().items():
            if key == "TYPE":
                if val.upper() not in ("3DBLOCK", "3DSTREAM"):
                    raise DescriptorError(f"line {ln}: TYPE {val} is not supported (3DBLOCK or 3DSTREAM)")
                k.type = val.upper()
            elif key == "STENCIL":
                k.stencil = _ints(val, 6, ln, "STENCIL")
                if any(h < 0 or h > 1 for h in k.stencil):
                    raise DescriptorError(f"line {ln}: STENCIL halos must be 0 or 1 (one ghost layer)")
            elif key == "TILE":
                k.tile = _ints(val, 3, ln, "TILE")
                tx, ty, tz = k.tile
                if tx % 64 or tx <= 0 or ty <= 0 or tz <= 0 or tx * ty > 1024:
                    raise DescriptorError(f"line {ln}: TILE x must be a multiple of 64, x*y <= 1024")
            else:
                raise DescriptorError(f"line {ln}: unknown kernel attribute {key}")
        self.take("{")
        while self.peek()[1] in ("VARIABLE", "PARAMETER"):
            if self.peek()[1] == "VARIABLE":
                attrs, names, group, ln = self.block("VARIABLE")
                v = Variable(names=names, group=group, line=ln)
                for key, (val, aln) in attrs.items():
                    val = val.upper()
                    if key == "CACHED":
                        v.cached = _yes(val, aln, key)
                    elif key == "INTENT":
                        if val not in INTENTS:
                            raise DescriptorError(f"line {aln}: INTENT {val} (one of {', '.join(INTENTS)})")
                        v.intent = val
                    elif key == "STORAGE":
                        if val not in ("FIELD", "FP64"):
                            raise DescriptorError(f"line {aln}: STORAGE {val} (FIELD or FP64)")
                        v.fp64 = val == "FP64"
                    elif key == "OPTIONAL":
                        v.optional = _yes(val, aln, key)
                    else:
                        raise DescriptorError(f"line {aln}: unknown variable attribute {key}")
                if v.cached and v.intent in ("OUT", "INOUT"):
                    raise DescriptorError(f"line {ln}: a cached variable is read only (IN or SEPARATEINOUT)")
                if v.optional and v.intent != "IN":
                    raise DescriptorError(f"line {ln}: only IN variables may be optional")
                k.variables.append(v)
            else:
                attrs, names, group, ln = self.block("PARAMETER")
                p = Parameter(names=names, group=group, line=ln)
                for key, (val, aln) in attrs.items():
                    if key == "SOURCE":
                        if val.upper() not in ("VALUE", "CONTROL"):
                            raise DescriptorError(f"line {aln}: SOURCE {val} (VALUE or CONTROL)")
                        p.control = val.upper() == "CONTROL"
                    else:
                        raise DescriptorError(f"line {aln}: unknown parameter attribute {key}")
                k.parameters.append(p)
        self.take("}")
        seen = set()
        for n in [n for n, _ in k.all_vars()] + [n for p in k.parameters for n in p.names]:
            if n in seen:
                raise DescriptorError(f"line {line}: {n} declared twice in kernel {k.name}")
            seen.add(n)
        return k

    def file(self):
        out = []
        while self.peek()[0] != "EOF":
            out.append(self.kernel())
        names = [k.name for k in out]
        if len(set(names)) != len(names):
            raise DescriptorError("a kernel name is declared twice")
        return out


def _ints(val, n, line, what):
    try:
        xs = tuple(int(x) for x in val.split(","))
    except ValueError:
        raise DescriptorError(f"line {line}: {what} must be {n} comma-separated integers") from None
    if len(xs) != n:
        raise DescriptorError(f"line {line}: {what} must have {n} entries")
    return xs


def _yes(val, line, what):
    if val not in ("YES", "NO"):
        raise DescriptorError(f"line {line}: {what} must be YES or NO")
    return val == "YES"


def parse(text: str) -> list:
    """Descriptor text -> list of Kernel records (DescriptorError with the
    line number on malformed input)."""
    return _Parser(text).file()


# ---- generator ----------------------------------------------------------------

def _storage(v):
    return "double" if v.fp64 else "T"


def generate(k: Kernel) -> str:
    """HIP header of one kernel (3DBLOCK template)."""
    tx, ty, tz = k.tile
    xm, xp, ym, yp, zm, zp = k.stencil
    lx, ly, lz = tx + xm + xp, ty + ym + yp, tz + zm + zp
    opt = k.optional_groups()
    tparams = "class T" + "".join(f", bool HAS_{g}" for g in opt)
    targs = "T" + "".join(f", HAS_{g}" for g in opt)
    body_file = f"bodies/{k.name.lower()}.h"
    L = []
    w = L.append
    w(f"// gen_{k.name.lower()}.h -- generated by descriptors/ccl.py from the descriptor of {k.name};")
    w("// do not edit (rebuilt by every build).")
    w(f"// TYPE={k.type} STENCIL=\"{','.join(map(str, k.stencil))}\" TILE=\"{tx},{ty},{tz}\"")
    w("#pragma once")
    w("")
    w("#include <hip/hip_runtime.h>")
    w("")
    w('#include "ns_internal.h"')
    w("")
    w("namespace ns {")
    w("namespace gen {")
    w("")
    # context: accessors for the body
    w(f"// What the body of {k.name} sees of its cell: position, accessors of")
    w("// the declared variables at an offset (di, dj, dk), stores, parameters.")
    w(f"template <{tparams}>")
    w(f"struct {k.name}_ctx {{")
    w("  const Geo& g;")
    w("  int i, j, k;  // 1-based cell indices")
    w("  long c;       // linear index in the padded layout")
    stream = k.type == "3DSTREAM"
    nplanes = zm + 1 + zp
    if stream:
        w("  int li;       // position of the cell in an LDS plane")
        w(f"  int pl[{nplanes}];    // LDS offset of planes k - {zm} .. k + {zp} in the ring")
    else:
        w("  int li;       // position of the cell in the LDS box")
    for n, v in k.all_vars():
        st = _storage(v)
        if v.cached:
            w(f"  const {st}* s_{n};  // {'LDS plane ring' if stream else 'LDS box'}")
        if v.intent in ("IN", "INOUT"):
            w(f"  {'const ' if v.intent == 'IN' else ''}{st}* __restrict__ {n}_p;")
        elif v.intent == "OUT":
            w(f"  {st}* __restrict__ {n}_p;")
        else:
            w(f"  const {st}* __restrict__ {n}_in_p;")
            w(f"  {st}* __restrict__ {n}_out_p;")
    for p in k.parameters:
        for n in p.names:
            w(f"  double {n};")
    for g in opt:
        w(f"  static constexpr bool has_{g} = HAS_{g};")
    for n, v in k.all_vars():
        st = _storage(v)
        rd = n if v.intent in ("IN", "INOUT") else (f"{n}_in" if v.intent == "SEPARATEINOUT" else None)
        if rd is not None:
            if v.cached and stream:
                w(f"  __device__ __forceinline__ {st} {rd}(int di = 0, int dj = 0, int dk = 0) const {{")
                w(f"    return s_{n}[pl[dk + {zm}] + li + dj * {lx} + di];")
                w("  }")
            elif v.cached:
                w(f"  __device__ __forceinline__ {st} {rd}(int di = 0, int dj = 0, int dk = 0) const {{")
                w(f"    return s_{n}[li + (dk * {ly} + dj) * {lx} + di];")
                w("  }")
            else:
                src = f"{n}_p" if v.intent != "SEPARATEINOUT" else f"{n}_in_p"
                w(f"  __device__ __forceinline__ {st} {rd}(int di = 0, int dj = 0, int dk = 0) const {{")
                w(f"    return {src}[c + di + dj * g.sx + dk * g.sxy];")
                w("  }")
        if v.intent in ("OUT", "INOUT"):
            w(f"  __device__ __forceinline__ void store_{n}(double x) const {{ {n}_p[c] = {st}(x); }}")
        elif v.intent == "SEPARATEINOUT":
            w(f"  __device__ __forceinline__ void store_{n}(double x) const {{ {n}_out_p[c] = {st}(x); }}")
    w("};")
    w("")
    w("}  // namespace gen")
    w("}  // namespace ns")
    w("")
    w(f'#include "{body_file}"')
    w("")
    w("namespace ns {")
    w("namespace gen {")
    w("")
    # kernel arguments
    args = []
    for n, v in k.all_vars():
        st = _storage(v)
        if v.intent == "IN":
            args.append(f"const {st}* __restrict__ {n}")
        elif v.intent in ("OUT", "INOUT"):
            args.append(f"{st}* __restrict__ {n}")
        else:
            args.append(f"const {st}* __restrict__ {n}_in")
            args.append(f"{st}* __restrict__ {n}_out")
    vals = [n for p in k.parameters if not p.control for n in p.names]
    args += [f"double {n}" for n in vals]
    cached = [(n, v) for n, v in k.all_vars() if v.cached]
    if stream:
        _stream_kernel(k, w, tparams, targs, args, cached, lx, ly, nplanes)
    else:
        _block_kernel(k, w, tparams, targs, args, cached, lx, ly, lz)
    _launcher(k, w, vals, opt)
    return "\n".join(L)


def _set_ctx(k, w, targs):
    w(f"  {k.name}_ctx<{targs}> x{{g}};")
    for n, v in k.all_vars():
        if v.cached:
            w(f"  x.s_{n} = s_{n};")
        if v.intent in ("IN", "OUT", "INOUT"):
            w(f"  x.{n}_p = {n};")
        else:
            w(f"  x.{n}_in_p = {n}_in;")
            w(f"  x.{n}_out_p = {n}_out;")
    for p in k.parameters:
        for n in p.names:
            w(f"  x.{n} = {'ctl->' + n if p.control else n};")


def _stream_kernel(k, w, tparams, targs, args, cached, lx, ly, nplanes):
    tx, ty, tz = k.tile
    xm, xp, ym, yp, zm, zp = k.stencil
    nthr = tx * ty
    plane = lx * ly
    per = (plane + nthr - 1) // nthr
    w(f"// One {tx} x {ty} tile of {k.name} per workgroup ({tx} x {ty} threads), marching")
    w(f"// {tz} planes; cached variables in a ring of {nplanes} LDS planes of {lx} x {ly}.")
    w(f"template <{tparams}>")
    w(f"__global__ void __launch_bounds__({nthr})")
    w(f"k_{k.name}(Geo g, const Ctl* __restrict__ ctl{''.join(', ' + a for a in args)}) {{")
    for n, v in cached:
        w(f"  __shared__ {_storage(v)} s_{n}[{nplanes * plane}];")
    w(f"  const int i0 = blockIdx.x * {tx} + 1, j0 = blockIdx.y * {ty} + 1;")
    w(f"  const int k0 = blockIdx.z * {tz} + 1, k1 = min(g.nz, k0 + {tz - 1});")
    w(f"  const int tid = threadIdx.x + {tx} * threadIdx.y;")
    if cached:
        w("  // this thread's entries of a staged plane (x fastest, positions clamped to")
        w("  // the padded array: clamped entries only feed cells outside the domain)")
        w(f"  long qo[{per}];")
        w(f"  bool qv[{per}];")
        w(f"#pragma unroll")
        w(f"  for (int r = 0; r < {per}; r++) {{")
        w(f"    const int t = tid + r * {nthr};")
        w(f"    qv[r] = t < {plane};")
        w(f"    const int gi = min(max(i0 - {xm} + t % {lx}, 0), g.nx + 1);")
        w(f"    const int gj = min(max(j0 - {ym} + t / {lx}, 0), g.ny + 1);")
        w("    qo[r] = (long)gj * g.sx + gi;")
        w("  }")
        w(f"  // planes k0 - {zm} .. k0 + {zp}; plane kk sits in ring slot kk % {nplanes}")
        w(f"  for (int d = -{zm}; d <= {zp}; d++) {{")
        w("    const long kk = min(k0 + d, g.nz + 1);")
        w(f"    const int sl = ((k0 + d) % {nplanes}) * {plane};")
        w(f"#pragma unroll")
        w(f"    for (int r = 0; r < {per}; r++)")
        w("      if (qv[r]) {")
        for n, v in cached:
            src = n if v.intent != "SEPARATEINOUT" else f"{n}_in"
            w(f"        s_{n}[sl + tid + r * {nthr}] = {src}[kk * g.sxy + qo[r]];")
        w("      }")
        w("  }")
        w("  __syncthreads();")
    _set_ctx(k, w, targs)
    w("  x.i = i0 + (int)threadIdx.x;")
    w("  x.j = j0 + (int)threadIdx.y;")
    w("  const bool act = x.i <= g.nx && x.j <= g.ny;")
    w(f"  x.li = ((int)threadIdx.y + {ym}) * {lx} + (int)threadIdx.x + {xm};")
    w("  for (int k = k0; k <= k1; k++) {")
    if cached:
        w("    const bool more = k < k1;  // the same in every thread")
        w(f"    const int kn = k + {zp + 1};  // the plane staged during this step")
        for n, v in cached:
            w(f"    {_storage(v)} pre_{n}[{per}];")
        w("    if (more) {")
        w("      const long kk = min(kn, g.nz + 1);")
        w(f"#pragma unroll")
        w(f"      for (int r = 0; r < {per}; r++) {{")
        for n, v in cached:
            src = n if v.intent != "SEPARATEINOUT" else f"{n}_in"
            w(f"        pre_{n}[r] = qv[r] ? {src}[kk * g.sxy + qo[r]] : {_storage(v)}(0);")
        w("      }")
        w("    }")
    w("    if (act) {")
    w("      x.k = k;")
    w("      x.c = (long)k * g.sxy + (long)x.j * g.sx + x.i;")
    if cached:
        w(f"#pragma unroll")
        w(f"      for (int d = 0; d < {nplanes}; d++) x.pl[d] = ((k - {zm} + d) % {nplanes}) * {plane};")
    w(f"      {k.name}_body(x);")
    w("    }")
    if cached:
        w("    if (more) {")
        w(f"      __syncthreads();  // every read of plane k - {zm} is done")
        w(f"      const int sl = (kn % {nplanes}) * {plane};")
        w(f"#pragma unroll")
        w(f"      for (int r = 0; r < {per}; r++)")
        w("        if (qv[r]) {")
        for n, v in cached:
            w(f"          s_{n}[sl + tid + r * {nthr}] = pre_{n}[r];")
        w("        }")
        w("      __syncthreads();")
        w("    }")
    w("  }")
    w("}")
    w("")


def _block_kernel(k, w, tparams, targs, args, cached, lx, ly, lz):
    tx, ty, tz = k.tile
    xm, xp, ym, yp, zm, zp = k.stencil
    w(f"// One {tx} x {ty} x {tz} tile of {k.name} per workgroup ({tx} x {ty} threads).")
    w(f"template <{tparams}>")
    w(f"__global__ void __launch_bounds__({tx * ty})")
    w(f"k_{k.name}(Geo g, const Ctl* __restrict__ ctl{''.join(', ' + a for a in args)}) {{")
    for n, v in cached:
        w(f"  __shared__ {_storage(v)} s_{n}[{lx * ly * lz}];")
    w(f"  const int i0 = blockIdx.x * {tx} + 1, j0 = blockIdx.y * {ty} + 1, k0 = blockIdx.z * {tz} + 1;")
    w(f"  const int tid = threadIdx.x + {tx} * threadIdx.y;")
    if cached:
        w("  // the cached variables' box: tile plus halo, x fastest, clamped to the")
        w("  // padded array (clamped entries only feed cells outside the domain)")
        w(f"  for (int t = tid; t < {lx * ly * lz}; t += {tx * ty}) {{")
        w(f"    const int a = t % {lx}, b = (t / {lx}) % {ly}, d = t / {lx * ly};")
        w(f"    const int gi = min(max(i0 - {xm} + a, 0), g.nx + 1);")
        w(f"    const int gj = min(max(j0 - {ym} + b, 0), g.ny + 1);")
        w(f"    const int gk = min(max(k0 - {zm} + d, 0), g.nz + 1);")
        w("    const long q = (long)gk * g.sxy + (long)gj * g.sx + gi;")
        for n, v in cached:
            src = n if v.intent != "SEPARATEINOUT" else f"{n}_in"
            w(f"    s_{n}[t] = {src}[q];")
        w("  }")
        w("  __syncthreads();")
    _set_ctx(k, w, targs)
    w("  x.i = i0 + (int)threadIdx.x;")
    w("  x.j = j0 + (int)threadIdx.y;")
    w("  if (x.i > g.nx || x.j > g.ny) return;")
    w(f"  for (int kz = 0; kz < {tz}; kz++) {{")
    w("    x.k = k0 + kz;")
    w("    if (x.k > g.nz) break;")
    w("    x.c = (long)x.k * g.sxy + (long)x.j * g.sx + x.i;")
    w(f"    x.li = ((kz + {zm}) * {ly} + (int)threadIdx.y + {ym}) * {lx} + (int)threadIdx.x + {xm};")
    w(f"    {k.name}_body(x);")
    w("  }")
    w("}")
    w("")


def _launcher(k, w, vals, opt):
    tx, ty, tz = k.tile
    largs = []
    for n, v in k.all_vars():
        st = _storage(v)
        if v.intent == "IN":
            largs.append((f"const {st}* {n}", n))
        elif v.intent in ("OUT", "INOUT"):
            largs.append((f"{st}* {n}", n))
        else:
            largs.append((f"const {st}* {n}_in", f"{n}_in"))
            largs.append((f"{st}* {n}_out", f"{n}_out"))
    largs += [(f"double {n}", n) for n in vals]
    w(f"// Launch over every interior cell of a domain; optional variable groups")
    w(f"// are present when their first pointer is not null.")
    w("template <class T>")
    w(f"hipError_t launch_{k.name}(hipStream_t st, const Geo& g, const Ctl* ctl"
      f"{''.join(', ' + a for a, _ in largs)}) {{")
    w(f"  const dim3 grid((g.nx + {tx - 1}) / {tx}, (g.ny + {ty - 1}) / {ty}, (g.nz + {tz - 1}) / {tz});")
    w(f"  const dim3 blk({tx}, {ty});")
    call_args = "g, ctl" + "".join(", " + n for _, n in largs)
    # dispatch over the optional groups
    def emit(idx, flags, indent):
        if idx == len(opt):
            ta = "T" + "".join(f", {'true' if f else 'false'}" for f in flags)
            w(f"{indent}k_{k.name}<{ta}><<<grid, blk, 0, st>>>({call_args});")
            return
        first = next(v.names[0] for v in k.variables if v.group == opt[idx])
        w(f"{indent}if ({first}) {{")
        emit(idx + 1, flags + [True], indent + "  ")
        w(f"{indent}}} else {{")
        emit(idx + 1, flags + [False], indent + "  ")
        w(f"{indent}}}")
    emit(0, [], "  ")
    w("  return hipGetLastError();")
    w("}")
    w("")
    w("}  // namespace gen")
    w("}  // namespace ns")
    w("")


def build(descriptor: str, out_dir: str) -> list:
    """Parse ``descriptor`` and write gen_<kernel>.h into ``out_dir`` (only
    files whose content changed are rewritten).  Returns the paths."""
    with open(descriptor) as fh:
        kernels = parse(fh.read())
    os.makedirs(out_dir, exist_ok=True)
    paths = []
    for k in kernels:
        path = os.path.join(out_dir, f"gen_{k.name.lower()}.h")
        text = generate(k)
        old = None
        if os.path.exists(path):
            with open(path) as fh:
                old = fh.read()
        if old != text:
            with open(path + ".tmp", "w") as fh:
                fh.write(text)
            os.replace(path + ".tmp", path)
        paths.append(path)
    return paths


DESCRIPTOR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kernels.ccl")

if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.getcwd(), "gen")
    for p in build(DESCRIPTOR, out):
        print(p)
