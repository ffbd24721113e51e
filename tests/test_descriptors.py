"""The kernel-descriptor layer on the CPU: the descriptor file parses into
the declared kernels, malformed descriptors are rejected with the line of
the mistake, and the generator's output is deterministic and carries the
declared tile, halo, variables and parameters."""
import os

import pytest

from paper_1201_2118_amd.descriptors import ccl


def _kernels():
    with open(ccl.DESCRIPTOR) as fh:
        return {k.name: k for k in ccl.parse(fh.read())}


def test_descriptor_file_declares_the_two_stencil_kernels():
    ks = _kernels()
    assert set(ks) == {"UPDATE_VELOCITY", "PREDICT_VELOCITY"}
    uv = ks["UPDATE_VELOCITY"]
    assert uv.type == "3DBLOCK" and uv.stencil == (0, 1, 0, 1, 0, 1) and uv.tile == (64, 4, 4)
    vel, pres = uv.variables
    assert vel.names == ["u", "v", "w"] and vel.intent == "SEPARATEINOUT" and not vel.cached
    assert pres.names == ["p"] and pres.intent == "IN" and pres.cached and pres.fp64
    assert [(p.names, p.control) for p in uv.parameters] == [(["dt"], True)]
    pv = ks["PREDICT_VELOCITY"]
    assert pv.type == "3DSTREAM" and pv.stencil == (1,) * 6 and pv.tile == (64, 8, 32)
    assert [(v.names, v.intent, v.cached, v.optional) for v in pv.variables] == [
        (["u", "v", "w"], "IN", True, False), (["F", "G", "H"], "OUT", False, False),
        (["fx", "fy", "fz"], "IN", False, True)]
    assert pv.optional_groups() == ["BODY_FORCE"]


BASE = """KERNEL K
  TYPE=3DBLOCK STENCIL="1,1,0,0,1,1" TILE="64,2,8"
{
  VARIABLE CACHED=YES INTENT=IN { a } "A"
  VARIABLE INTENT=OUT { b } "B"
  PARAMETER { s } "S"
}
"""


@pytest.mark.parametrize("edit,line,msg", [
    (("INTENT=OUT", "INTENT=SIDEWAYS"), 5, "INTENT SIDEWAYS"),
    (('STENCIL="1,1,0,0,1,1"', 'STENCIL="2,1,0,0,1,1"'), 2, "0 or 1"),
    (('TILE="64,2,8"', 'TILE="48,2,8"'), 2, "multiple of 64"),
    (('TILE="64,2,8"', 'TILE="64,2"'), 2, "3 entries"),
    (("TYPE=3DBLOCK", "TYPE=2DPLANE"), 2, "not supported"),
    (("TYPE=3DBLOCK", "TYPE=3DSTREAMS"), 2, "not supported"),
    (("VARIABLE INTENT=OUT { b }", "VARIABLE CACHED=YES INTENT=OUT { b }"), 5, "read only"),
    (("PARAMETER { s }", "PARAMETER { a }"), 1, "declared twice"),
    (("PARAMETER { s }", "PARAMETER SOURCE=HOST { s }"), 6, "SOURCE HOST"),
    (('{ b } "B"', '{ b "B"'), 5, "expected '}'"),
    (("CACHED=YES INTENT=IN", "CACHED=MAYBE INTENT=IN"), 4, "YES or NO"),
    (('"S"\n}', '"S"\n'), 8, "expected '}'"),
    (("{ a }", "{ a; }"), 4, "unexpected character"),
])
def test_malformed_descriptors_name_the_line(edit, line, msg):
    text = BASE.replace(*edit)
    assert text != BASE
    with pytest.raises(ccl.DescriptorError) as e:
        ccl.parse(text)
    assert f"line {line}:" in str(e.value) and msg in str(e.value), str(e.value)


def test_generated_header_carries_the_declarations():
    (k,) = ccl.parse(BASE)
    src = ccl.generate(k)
    # tile of 64 x 2 threads, LDS box (64+2) x 2 x (8+2) for the cached variable
    assert "__launch_bounds__(128)" in src
    assert "s_a[1320]" in src
    assert "k_K(Geo g, const Ctl* __restrict__ ctl, const T* __restrict__ a, T* __restrict__ b, double s)" in src
    assert "store_b(double x)" in src and '#include "bodies/k.h"' in src
    assert ccl.generate(k) == src  # deterministic


def test_stream_header_rings_the_planes_the_stencil_reaches():
    """3DSTREAM: a ring of z- + 1 + z+ LDS planes of (x + x- + x+) x (y + y- +
    y+) entries per cached variable; planes k0 - z- .. k0 + z+ staged first;
    at step k the plane k + z+ + 1 loads into registers and, between two
    barriers, replaces plane k - z- (slot kn % ring); the accessor reads plane
    k + dk from the ring slot of (k - z- + (dk + z-)) % ring."""
    for zm, zp, ring in ((1, 1, 3), (0, 1, 2), (1, 0, 2), (0, 0, 1)):
        text = BASE.replace('TYPE=3DBLOCK STENCIL="1,1,0,0,1,1"', f'TYPE=3DSTREAM STENCIL="1,1,0,0,{zm},{zp}"')
        (k,) = ccl.parse(text)
        src = ccl.generate(k)
        plane = (64 + 2) * 2
        assert f"s_a[{ring * plane}]" in src, (zm, zp)
        assert f"for (int d = -{zm}; d <= {zp}; d++)" in src
        assert f"const int kn = k + {zp + 1};" in src
        assert f"const int sl = (kn % {ring}) * {plane};" in src
        assert f"x.pl[d] = ((k - {zm} + d) % {ring}) * {plane};" in src
        assert f"return s_a[pl[dk + {zm}] + li + dj * 66 + di];" in src
        assert src.count("__syncthreads();") == 3  # after the first planes, around the refill
        # the slot schedule: at every step the ring holds planes k - zm .. k + zp
        for k0, k1 in ((1, 8), (5, 5), (3, 11)):
            slots = {(k0 + d) % ring: k0 + d for d in range(-zm, zp + 1)}
            for kk in range(k0, k1 + 1):
                for d in range(ring):
                    assert slots[(kk - zm + d) % ring] == kk - zm + d
                if kk < k1:
                    kn = kk + zp + 1
                    assert slots[kn % ring] == kk - zm  # the plane it replaces is no longer read
                    slots[kn % ring] = kn


def test_build_writes_one_header_per_kernel(tmp_path):
    paths = ccl.build(ccl.DESCRIPTOR, str(tmp_path))
    assert sorted(os.path.basename(p) for p in paths) == ["gen_predict_velocity.h", "gen_update_velocity.h"]
    for p in paths:
        src = open(p).read()
        assert "generated by descriptors/ccl.py" in src
    mt = [os.path.getmtime(p) for p in paths]
    ccl.build(ccl.DESCRIPTOR, str(tmp_path))  # unchanged content is not rewritten
    assert [os.path.getmtime(p) for p in paths] == mt
