"""Issue order of the block copies in the fused pass kernels' gfx950 code (host only).

The pair-tile and FP64 pass kernels stream their factor blocks into LDS with
global -> LDS loads and enter the first stage with a counted wait: at most
``pending + state loads`` vector-memory operations may still be outstanding, which
releases the first stage's copies only if they were issued before the tile's state
loads and the later stages' copies (loads complete in issue order).  The compiler is
free to interleave independent loads, so this order is checked here on the
compiled code: the pass kernels are compiled to gfx950 assembly, each one's
vector-memory loads up to the first barrier are replayed against its waits, and
the first stage's copies must all have completed when the barrier is reached.
"""
import concurrent.futures
import os
import re
import shutil
import subprocess

import pytest

from paper_1502_01379_amd import build as bfbuild

pytestmark = pytest.mark.slow

CSRC = bfbuild.CSRC


def _define(path, name):
    m = re.search(rf"#define {name} (\d+)", open(path).read())
    assert m, name
    return int(m.group(1))


def _compile(src, out_dir):
    out = os.path.join(out_dir, os.path.basename(src).replace(".hip", ".s"))
    cmd = [bfbuild.HIPCC, *bfbuild.DEVICE_FLAGS, "--cuda-device-only", "-S", "-I", bfbuild.INCLUDE,
           "-I", CSRC, src, "-o", out]
    cmd = [c for c in cmd if c not in ("-fPIC", "-c")]
    subprocess.run(cmd, check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return open(out).read()


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if shutil.which(bfbuild.HIPCC) is None and not os.path.exists(bfbuild.HIPCC):
        pytest.skip("hipcc not available")
    d = str(tmp_path_factory.mktemp("asm"))
    srcs = [os.path.join(CSRC, f) for f in ("bf_fused_f64.hip", "bf_fused_f32.hip", "bf_fused_bf16.hip")]
    with concurrent.futures.ThreadPoolExecutor(3) as ex:
        return dict(zip(("f64", "f32", "bf16"), ex.map(lambda s: _compile(s, d), srcs)))


def _kernels(text, pattern):
    """(template arguments, body) of every kernel whose symbol matches pattern."""
    parts = re.split(r"\n(_Z[^\s:]*):", text)
    for name, body in zip(parts[1::2], parts[2::2]):
        m = re.search(pattern, name)
        if m:
            yield tuple(int(x) for x in m.groups()), body.split("\n")


def _replay(lines, first_stage):
    """Replay the vector-memory loads from the first copy to the point where the first
    stage is read (the first barrier, or the first LDS read where the workgroup is one
    wavefront and the compiler drops its barriers), on every path through the branches
    in between (uniform address selects, the middle level's scaling loads).  Loads
    complete in issue order, so s_waitcnt vmcnt(n) leaves the last n outstanding.
    Returns the issue orders seen ("L" copy, "g" other load) and the first-stage copies
    still outstanding on some path."""
    ins = [l.strip() for l in lines]
    labels = {s[:-1]: i for i, s in enumerate(ins) if re.match(r"^\.LBB\w+:$", s)}
    start = next(i for i, s in enumerate(ins) if s.startswith("global_load_lds"))
    orders, late, seen = set(), set(), set()
    work = [(start, (), "", 0)]
    while work:
        i, outstanding, order, ncopy = work.pop()
        while True:
            if (i, outstanding, order) in seen:
                break
            seen.add((i, outstanding, order))
            s = ins[i]
            assert len(order) < 400 and not s.startswith("s_endpgm"), "no barrier on some path"
            if s.startswith(("s_barrier", "ds_read")):
                orders.add(order)
                late.update(c for c in outstanding if c[0] == "L" and c[1] < first_stage)
                break
            if s.startswith("global_load"):
                tag = ("L", ncopy) if s.startswith("global_load_lds") else ("g", len(order))
                ncopy += tag[0] == "L"
                outstanding, order = outstanding + (tag,), order + tag[0]
            elif s.startswith("s_waitcnt") and "vmcnt" in s:
                n = int(re.search(r"vmcnt\((\d+)\)", s).group(1))
                outstanding = outstanding[max(0, len(outstanding) - n):]
            elif s.startswith("s_branch"):
                i = labels[s.split()[1]]
                continue
            elif s.startswith("s_cbranch"):
                work.append((labels[s.split()[1]], outstanding, order, ncopy))
            i += 1
    return orders, sorted(late)


def test_f64_first_stage_copies_complete_at_first_barrier(asm):
    seen = 0
    pattern = r"k_fused_pass_f64ILi(\d)ELb(\d)ELb(\d)ELi(\d)ELi(\d)ELi(\d)E"
    for (K, li, lo, cw, nbuf, parts), lines in _kernels(asm["f64"], pattern):
        first = (8 if li else 16) // parts // cw  # 1 KB pieces of the first stage per wavefront
        orders, late = _replay(lines, first)
        assert all(o.startswith("L" * first) for o in orders), (K, li, lo, cw, orders)
        assert not late, f"K={K} LI={li} LO={lo} CW={cw}: first-stage copies {late} outstanding ({orders})"
        seen += 1
    assert seen == 24  # K = 1 .. 4, leaf-in / middle / leaf-out, one or two chunks per workgroup


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_pair_tile_first_stage_copies_complete_at_first_barrier(asm, prec):
    pb = _define(os.path.join(CSRC, "bf_fused_kernel.h"), "BF_SPLIT_PB")
    seen = 0
    pattern = r"k_fused_pass_x2ILi(\d)ELi(\d)ELb(\d)ELb(\d)ELi(\d)ELb(\d)E"
    for (K, p, li, lo, cp, io), lines in _kernels(asm[prec], pattern):
        wb = (1 << (K - 1)) // 2
        first = 2 * min(wb, pb) * (4 if li else 8) // (2 * cp)  # 1 KB pieces of the first stage per wavefront
        orders, late = _replay(lines, first)
        assert all(o.startswith("L" * first) for o in orders), (K, li, lo, cp, orders)
        assert not late, f"K={K} LI={li} LO={lo} CP={cp}: first-stage copies {late} outstanding ({orders})"
        seen += 1
    assert seen >= 24


def _barrier_model(K, li, lo, wb, parts, copies, two_waves):
    """Per-wavefront copies of each stage and the kinds of the barriers in program
    order (a stage index, or None for the barriers of the half-swap before the last
    level), for a pass of K levels with wb blocks per wavefront per level."""
    groups = (1 if li else 0) + K + (1 if lo else 0)
    per_group = wb * parts
    nst = groups * per_group
    cps = [copies(s // per_group in ((0,) if li else ()) or (lo and s // per_group == groups - 1)) for s in range(nst)]
    if not two_waves:
        return cps, list(range(nst))
    gl = (1 if li else 0) + K - 1  # group of the last level, entered after the swap
    return cps, list(range(gl * per_group)) + [None] * (2 * wb - 1) + list(range(gl * per_group, nst))


def _replay_stages(lines, cps, barriers):
    """Walk every path from the kernel entry to its end; at each stage barrier no copy
    of that stage or an earlier one may be outstanding.  Copies issued before the first
    other load (the first stage's blocks, and the middle weights where a pass stages
    them with it) belong to the first stage.  Returns the violations and the (barriers,
    copies before the state loads, copies after) counts seen at the end of each path."""
    stage = [s for s, c in enumerate(cps) for _ in range(c)]
    ins = [l.strip() for l in lines]
    labels = {s[:-1]: i for i, s in enumerate(ins) if re.match(r"^\.LBB\w+:$", s)}
    bad, ends, seen = set(), set(), set()
    work = [(0, (), 0, 0, 0, False)]
    while work:
        i, outstanding, ncopy, nfirst, nbar, state = work.pop()
        while True:
            key = (i, outstanding, ncopy, nfirst, nbar, state)
            if key in seen:
                break
            seen.add(key)
            s = ins[i]
            if s.startswith("s_endpgm"):
                # no global -> LDS copy may land after the workgroup has ended
                if any(c != "g" for c in outstanding):
                    bad.add(("copies outstanding at the end", nbar))
                ends.add((nbar, nfirst, ncopy))
                break
            if s.startswith("s_barrier"):
                kind = barriers[nbar] if nbar < len(barriers) else "extra"
                if kind == "extra":
                    bad.add(("extra barrier", nbar))
                elif kind is not None:
                    late = [0 if c < 0 else stage[c] for c in outstanding if c != "g" and (c < 0 or stage[c] <= kind)]
                    if late:
                        bad.add((kind, tuple(sorted(set(late)))))
                nbar += 1
            elif s.startswith("global_load"):
                if s.startswith("global_load_lds") and not state:
                    outstanding, nfirst = outstanding + (-1 - nfirst,), nfirst + 1
                elif s.startswith("global_load_lds"):
                    assert cps[0] + ncopy < len(stage), \
                        "more copies after the state loads than the later stages issue (a first-stage copy after a state load?)"
                    outstanding, ncopy = outstanding + (cps[0] + ncopy,), ncopy + 1
                else:
                    outstanding, state = outstanding + ("g",), True
            elif s.startswith("s_waitcnt") and "vmcnt" in s:
                n = int(re.search(r"vmcnt\((\d+)\)", s).group(1))
                outstanding = outstanding[max(0, len(outstanding) - n):]
            elif s.startswith("s_branch"):
                i = labels[s.split()[1]]
                continue
            elif s.startswith("s_cbranch"):
                work.append((labels[s.split()[1]], outstanding, ncopy, nfirst, nbar, state))
            i += 1
    return bad, ends


def test_f64_every_stage_copies_complete_at_its_barrier(asm):
    checked = 0
    pattern = r"k_fused_pass_f64ILi(\d)ELb(\d)ELb(\d)ELi(\d)ELi(\d)ELi(\d)E"
    for (K, li, lo, cw, nbuf, parts), lines in _kernels(asm["f64"], pattern):
        w = 2 if K >= 3 else 1
        if w * cw == 1:
            continue  # one wavefront per workgroup: no barriers (the first-stage test covers it)
        wb = (1 << K) // w // 2
        cps, barriers = _barrier_model(K, li, lo, wb, parts,
                                       lambda leaf: (8 if leaf else 16) // parts * w // (w * cw), w == 2)
        bad, ends = _replay_stages(lines, cps, barriers)
        assert not bad, f"K={K} LI={li} LO={lo} CW={cw}: {sorted(bad)[:4]}"
        # the passes after the middle level also stage the middle weights (one copy)
        expect = {(len(barriers), cps[0], sum(cps) - cps[0])}
        if not li:
            expect.add((len(barriers), cps[0] + 1, sum(cps) - cps[0]))
        assert ends == expect, (K, li, lo, cw, ends, expect)
        checked += 1
    assert checked == 18


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_pair_tile_every_stage_copies_complete_at_its_barrier(asm, prec):
    pb = _define(os.path.join(CSRC, "bf_fused_kernel.h"), "BF_SPLIT_PB")
    checked = 0
    pattern = r"k_fused_pass_x2ILi(\d)ELi(\d)ELb(\d)ELb(\d)ELi(\d)ELb(\d)E"
    for (K, p, li, lo, cp, io), lines in _kernels(asm[prec], pattern):
        wb = (1 << (K - 1)) // 2
        pbk = min(wb, pb)
        cps, barriers = _barrier_model(K, li, lo, wb // pbk, 1,
                                       lambda leaf: 2 * pbk * (4 if leaf else 8) // (2 * cp), True)
        bad, ends = _replay_stages(lines, cps, barriers)
        assert not bad, f"K={K} LI={li} LO={lo} CP={cp} IO={io}: {sorted(bad)[:4]}"
        if io:
            # a pass run only for the states inside it ends before the half-swap
            assert {e[0] for e in ends} == {barriers.index(None)}, (K, li, lo, cp, ends)
        else:
            assert ends == {(len(barriers), cps[0], sum(cps) - cps[0])}, (K, li, lo, cp, ends)
        checked += 1
    assert checked >= 24  # the full passes and the passes run only for their inner states
