# Profiling helper (not a test; run under rocprofv3 --pmc): one serial SY2SB n=16384 w=b=128 on a symmetric N(0,1) matrix (no QR in the input
# generation), preceded by a plain 2 GiB device copy used to calibrate the
# FETCH_SIZE / WRITE_SIZE counters
import sys
sys.path.insert(0, "/root/repo")
import torch
import paper_1709_00302_amd as br
br.load()
n = 16384
g = torch.Generator(device="cuda"); g.manual_seed(1)
Z = torch.randn(n, n, generator=g, device="cuda", dtype=torch.float64)
A = (torch.triu(Z) + torch.triu(Z, 1).T).T.contiguous().T
B = torch.empty_like(A)
torch.cuda.synchronize()
B.copy_(A)          # calibration: reads and writes n*n*8 bytes
torch.cuda.synchronize()
# the serial reduction (no look-ahead): its launches are the ones the bench's
# roofline figure covers (every kernel alone on the GPU)
tau = br.sy2sb(A, 128, 128, lookahead=False)
torch.cuda.synchronize()
print("done", float(tau[:4].sum()))
