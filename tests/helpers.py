"""Shared helpers for the test suite (fixture loading, OpenSSL known answers)."""
import csv
import os
import shutil
import subprocess
import tempfile

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    """Rows of a golden CSV (comment lines start with '#'), values as numbers."""
    path = os.path.join(GOLDEN, name)
    with open(path) as f:
        lines = [ln for ln in f if not ln.startswith("#")]
    rows = []
    for r in csv.DictReader(lines):
        rows.append({k: (float(v) if "." in v else int(v)) for k, v in r.items()})
    return rows


def have_openssl():
    return shutil.which("openssl") is not None


def openssl_params():
    """(p, a, b, Gx, Gy, q, cofactor) of prime256v1 as printed by OpenSSL."""
    out = subprocess.run(["openssl", "ecparam", "-name", "prime256v1", "-param_enc", "explicit",
                          "-text", "-noout"], check=True, capture_output=True, text=True).stdout
    fields = {}
    cur = None
    for line in out.splitlines():
        s = line.strip()
        head = s.split(":")[0]
        if head in ("Prime", "A", "B", "Generator (uncompressed)", "Order", "Cofactor", "Seed"):
            cur = head
            fields[cur] = ""
            rest = s[len(head) + 1:].strip()
            if cur == "Cofactor":
                fields[cur] = rest.split()[0]
                cur = None
            elif rest:
                fields[cur] += rest
            continue
        if cur and s and all(c in "0123456789abcdef:" for c in s):
            fields[cur] += s
    hexv = {k: v.replace(":", "") for k, v in fields.items()}
    gen = hexv["Generator (uncompressed)"]
    assert gen.startswith("04")
    gen = gen[2:]
    return (int(hexv["Prime"], 16), int(hexv["A"], 16), int(hexv["B"], 16), int(gen[:64], 16),
            int(gen[64:], 16), int(hexv["Order"], 16), int(fields["Cofactor"]))


def openssl_pubkey(k: int):
    """(x, y) of k*G on prime256v1 computed by OpenSSL from a raw private key."""
    with tempfile.TemporaryDirectory() as d:
        cnf = os.path.join(d, "k.cnf")
        der = os.path.join(d, "k.der")
        with open(cnf, "w") as f:
            f.write("asn1=SEQUENCE:ecpriv\n[ecpriv]\nversion=INTEGER:1\n")
            f.write("priv=FORMAT:HEX,OCTETSTRING:%064x\n" % k)
            f.write("params=EXPLICIT:0,OID:prime256v1\n")
        subprocess.run(["openssl", "asn1parse", "-genconf", cnf, "-out", der, "-noout"],
                       check=True, capture_output=True)
        out = subprocess.run(["openssl", "ec", "-inform", "DER", "-in", der, "-text", "-noout"],
                             check=True, capture_output=True, text=True).stdout
    hexs = ""
    take = False
    for line in out.splitlines():
        s = line.strip()
        if s.startswith("pub:"):
            take = True
            continue
        if take:
            if s and all(c in "0123456789abcdef:" for c in s):
                hexs += s.replace(":", "")
            else:
                break
    assert hexs.startswith("04"), out
    hexs = hexs[2:]
    return int(hexs[:64], 16), int(hexs[64:], 16)
