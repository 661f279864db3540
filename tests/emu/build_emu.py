"""Build libmcg_emu.so: the MCG library (driver and kernels, unchanged
sources) compiled as host C++20 against the emulated HIP runtime in
tests/emu/include, with AddressSanitizer and UBSan.  The kernel launches of
each k_*.hip launcher file are rewritten mechanically from
`K<<<grid, block, 0, s>>>(args)` to `EMU_LAUNCH((K), grid, block, s, args)`.
Test infrastructure only."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_0807_0264_amd", "csrc")
OUT = os.path.join(HERE, "_gen")
LIB = os.path.join(HERE, "libmcg_emu.so")


def _match_back(s, i):
    """start index of the kernel expression that ends just before s[i]"""
    j = i
    if s[j - 1] == ">":  # template arguments
        depth = 0
        while True:
            j -= 1
            if s[j] == ">":
                depth += 1
            elif s[j] == "<":
                depth -= 1
                if depth == 0:
                    break
    while j > 0 and (s[j - 1].isalnum() or s[j - 1] in "_:"):
        j -= 1
    return j


def _split_top(s):
    parts, depth, cur = [], 0, ""
    for ch in s:
        if ch in "(<[{":
            depth += 1
        elif ch in ")>]}":
            depth -= 1
        if ch == "," and depth == 0:
            parts.append(cur.strip())
            cur = ""
        else:
            cur += ch
    parts.append(cur.strip())
    return parts


def convert(src):
    out, pos = "", 0
    while True:
        i = src.find("<<<", pos)
        if i < 0:
            return out + src[pos:]
        k0 = _match_back(src, i)
        j = src.index(">>>", i)
        cfg = _split_top(src[i + 3:j])
        assert len(cfg) == 4 and cfg[2] == "0", cfg
        assert src[j + 3] == "("
        depth, m = 0, j + 3
        while True:
            if src[m] == "(":
                depth += 1
            elif src[m] == ")":
                depth -= 1
                if depth == 0:
                    break
            m += 1
        args = src[j + 4:m]
        out += src[pos:k0] + f"EMU_LAUNCH(({src[k0:i]}), {cfg[0]}, {cfg[1]}, {cfg[3]}, {args})"
        pos = m + 1


def build(verbose=False):
    os.makedirs(OUT, exist_ok=True)
    srcs = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".hip"):
            g = os.path.join(OUT, f[:-4] + "_emu.cpp")
            open(g, "w").write(convert(open(os.path.join(CSRC, f)).read()))
            srcs.append(g)
    srcs.append(os.path.join(CSRC, "mcg_api.cpp"))
    flags = ["g++", "-std=c++20", "-O1", "-g", "-fPIC", "-pthread",
             "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
             "-Wno-unknown-pragmas", "-Wno-attributes",
             "-I", os.path.join(HERE, "include"), "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    procs, objs = [], []
    for src in srcs:
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen(flags + ["-c", src, "-o", obj]))
    if any(p.wait() != 0 for p in procs):
        raise RuntimeError("emulation build failed")
    cmd = ["g++", "-shared", "-fsanitize=address,undefined", "-pthread", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
